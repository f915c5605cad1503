// Device code of the IPGC library: data layout, helpers, preparation kernels,
// the two per-round steps of IPGC (Section II-C of Rai, M P, Pai, "A Hybrid
// Graph Coloring Algorithm for GPUs", arXiv 1912.01478) and the round schedule
// of Section IV (a topology-driven sweep or a data-driven worklist pass, picked
// per round from the worklist size; the worklist is kept in both).
//
// Racy mode (optional): a loser writes 0 at once, so a later test in the same
// step no longer sees its color, and light nodes also avoid their neighbours'
// visible tentative colors.  The result depends on timing but is a proper
// coloring: the smallest active id still commits every round.
//
// Color state: one int32 per node in the caller's output buffer.
//   c[v] > 0   v holds committed color c[v];
//   c[v] <= 0  v is uncolored; after the assign step it holds -t (t >= 1 is its
//              tentative color of the round).
// Assign reads only c[u] > 0, so concurrent writes of -t are invisible to it.
// Conflict compares |c[u]| with the node's own tentative color: a neighbour
// that commits in the same step flips -t to +t, |c[u]| unchanged, and a
// neighbour committed in an earlier round holds a color that was forbidden to
// the node, so it never matches.  The result is the synchronous one whatever
// the timing, with no second state array.
//
// Byte maps: node v owns bytes [rowptr[v] + v, rowptr[v + 1] + v] of F, one
// per color 1..d+1; a byte is set once a neighbour has committed that color.
//
// A packed batch of graphs runs as one graph, the disjoint union: node ids are
// global (each graph's first id plus the local id), row offsets are 64-bit,
// and neighbour ids read from a row are shifted by the row owner's graph base.
// The lower id still decides every conflict inside a graph, so each graph gets
// exactly the coloring it gets alone; its round count is the last round in
// which one of its nodes committed.
//
// Node classes by degree d:
//   L (d <= light_max <= 32)  a thread per node.  Assign reads the row's colors
//                             into a 64-bit mask (the answer is at most d+1);
//                             conflict scans the row.
//   W (light_max < d <= hub)  a wavefront per node.  Forbidden colors live in a
//                             byte map F_v (one byte per color 1..d+1) that
//                             committing neighbours write into; assign scans
//                             F_v from the node's previous tentative color (the
//                             first free color never decreases, because
//                             committed colors never change).
//   M (d > hub)               as W, except that when an M node commits, the
//                             whole grid writes its color into its neighbours'
//                             byte maps in a separate step of the round (a
//                             hub's row is too long for one wavefront).
// Conflict scans of W/M nodes read a private list of the node's smaller
// neighbours (u < v) kept in a ring inside the node's CSR-sized region: each
// scan drops the neighbours it finds committed and moves the start past what
// it read, so every dead entry is read once after it dies and the scan
// position rotates through the list.
//
// Worklists are split into one segment per workgroup and class; a workgroup
// appends its losers to its own segments with shared-memory counters, so no
// global atomic is involved.  Readers map item numbers to segments with a
// prefix sum of the segment counts held in shared memory.
//
// Grid barrier (cooperative launch): workgroups run on the XCD given by their
// XCC_ID register.  The last workgroup of an XCD to arrive writes back that
// XCD's L2 (agent-scope release) once for all of them; the XCD leaders meet on
// a global counter; every workgroup then invalidates its caches (agent-scope
// acquire).  Before arriving, every thread waits until its stores have reached
// the L2, which all workgroups of the XCD share.
#pragma once

#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ipgc {

constexpr int kWave = 64;
constexpr int kPrepBlock = 256;
constexpr int kRoundBlock = 1024;        // 16 wavefronts; one workgroup per CU
constexpr int kRoundWaves = kRoundBlock / kWave;
constexpr int kMaxRoundBlocks = 1024;    // cap on the cooperative grid
constexpr int kLightMaxLimit = 32;       // thread-per-node pull uses a 64-bit mask: d + 1 <= 64
constexpr int kMaxXcc = 16;
constexpr int kWideScanMax = 65536;      // rounds with at most this many active nodes scan rings 4 chunks a pass
constexpr int kMaskColors = 64;          // colors 1..64 of committed neighbours are bits of a word per node
constexpr int kRingChunk = 2048;         // row entries of a class-M node whose ring part one wavefront builds
constexpr int kMaxSplitGraphs = 65536;   // per-graph schedules: graphs of a batch at most (a bit each in shared memory)

enum { kL = 0, kW = 1, kM = 2, kNumClasses = 3 };

// How committed colors reach the nodes of class L:
//   kPushAll   every winner writes its color into every neighbour's byte map;
//   kPullLight L nodes read their neighbours' colors in each assign (a register
//              mask: d + 1 <= 33 colors matter), winners write only into the maps
//              of W/M neighbours;
//   kPullOnly  as kPullLight on a graph with no W/M node: nobody writes maps.
enum { kPushAll = 0, kPullLight = 1, kPullOnly = 2 };

// Work counters (units for the algorithmic byte count).
enum {
    kUAssignNodes = 0,  // nodes given a tentative color
    kUPullEntries,      // row entries read by thread-per-node assigns
    kUMapBytes,         // byte-map bytes scanned by W/M assigns
    kUConflictNodes,    // nodes tested for conflicts
    kUConflictEntries,  // neighbour entries read by conflict scans
    kUListWrites,       // list entries kept and rewritten by W/M conflict scans
    kUPushEntries,      // row entries read by winners writing into neighbours' byte maps
    kUCommits,          // nodes committed
    kNumUnits
};

struct alignas(128) Line {
    unsigned v;
    unsigned pad[31];
};

struct Barrier {
    Line xcnt[kMaxXcc];   // arrivals per XCD
    Line xsize[kMaxXcc];  // workgroups per XCD
    Line gcnt;            // XCD leaders arrived
    Line gen;             // global generation
    Line xgen[kMaxXcc];   // generation released per XCD
    Line setup;           // one-time flat barrier counter
    Line abort;           // set by a workgroup whose wait exceeded the time limit: everyone leaves
    unsigned xcc_of[kMaxRoundBlocks];  // XCD of every workgroup (for a smaller set of participants)
};

// Scalars shared by every kernel of a call.
struct Counters {
    int64_t class_deg[kNumClasses];   // degree sum per class (static list)
    int64_t unit_nodes[4];            // active nodes per class summed over rounds
    int64_t unit_edges[4];            // their degree sums summed over rounds
    int32_t class_n[kNumClasses];     // nodes per class
    int64_t seg_off[4];               // class regions of the segmented lists
    int32_t static_off[4];            // class regions of the static list
    int32_t seg_cap[kNumClasses];     // entries per workgroup segment, per class
    int32_t finished;
    int32_t rounds;
    int32_t bad_rows;
    int32_t bad_ids;
    int32_t unsorted;
    int32_t hub_winners;              // hubs committed in the current round
    int32_t prev_discarded;           // the last round kept no worklist (discard mode, stepped launches)
    int32_t bad_full;                 // IPGC_VALIDATE_FULL: bit 0 self-loop, bit 1 duplicate, bit 2 no reverse entry
    int32_t seg_overflow;             // a workgroup had more losers than its out segment holds (never expected)
    int32_t hub_chunks;               // row chunks of kRingChunk entries over all class-M nodes
    int32_t static_ident;             // class L or W holds every node: its static list is 0, 1, ..., n-1 (not written)
    int32_t bad_ends;                 // rowptr[0] != 0 or rowptr[n] != m (their values in ends)
    int32_t split_topo;               // per-graph schedules, stepped launches: graphs with active nodes of
    int32_t split_data;               // each kind in the current round (written by its assign launch)
    int32_t resume_round;             // per-graph schedules: the round from which every graph runs data-driven,
                                      // left by the per-graph round kernel to the plain one (0: none)
    int64_t ends[2];
};

// True if the preparation kernels found the input unusable; the round kernels
// then run no round (every workgroup reads the same flags) and the host
// reports the error.
__device__ __forceinline__ bool input_bad(const Counters *ct) {
    return ct->bad_ends | ct->bad_rows | ct->bad_ids;
}

// A committed hub waiting for the push step.
struct HubRec {
    int64_t b, e;   // row entries
    int64_t fsh;    // byte-map shift of its graph
    int32_t t;      // its color
    int32_t base;   // first global id of its graph
};

// Everything a kernel needs, passed by value.  Off is the type of the row
// offsets: int32_t for one graph, int64_t for a packed batch of graphs, which
// the kernels see as one graph (the disjoint union) with global node ids.
template <typename Off, bool SPLIT = false>
struct DevT {
    using OffT = Off;
    static constexpr bool kSplit = SPLIT;  // per-graph schedules compiled in (batches only)
    const Off *rowptr;       // row starts, n + 1 entries (a batch: union row starts)
    const int32_t *colidx;   // column indices (a batch: ids local to each graph)
    const int32_t *gbase;    // a batch: first global id of each node's graph (null for one graph)
    const int32_t *gidx;     // a batch: graph index of each node (null for one graph)
    const int64_t *gend;     // a batch: one past the last global id of each graph
    int32_t *grounds;        // a batch: rounds per graph (the last round one of its nodes committed)
    int32_t *gleft;          // a server: uncommitted nodes per graph (null otherwise)
    const int64_t *gfshift;  // a server: byte-map shift per graph (null: no shift)
    int32_t *c;              // color state (caller's output)
    const int8_t *cls;       // class per node
    uint64_t *mask;          // per node: bit t - 1 set iff a committed neighbour has color t (t <= 64)
    uint32_t *pend;          // class L: bit j set while row entry j's neighbour has not been seen committed
    uint8_t *F;              // byte maps for colors above 64: node v's map is bytes [rowptr[v] + v,
                             // rowptr[v + 1] + v] (byte t - 1 for color t), shifted by fshift(v)
    int32_t *lower;          // ring of smaller neighbours per W/M node (region rowptr[v] .. + d)
    int32_t *lstart;         // ring start per node
    int32_t *llen;           // ring length per node
    int32_t *static_list;    // every node grouped by class (ascending id inside a class)
    int32_t *seg_list[2];    // the two alternating segmented worklists
    int32_t *seg_cnt[2];     // [kNumClasses][grid] entries per segment
    int64_t *seg_deg[2];     // [kNumClasses][grid] degree sum per segment
    HubRec *hub_won;         // hubs committed in the current round
    int32_t *block_cnt;      // [kNumClasses + 1][prep grid] class counts (then class-M row chunks) per
                             // preparation workgroup
    int32_t *hub_pre;        // class-M nodes in static-list order: first row chunk of each (+ the total)
    int32_t *hub_cnt;        // per row chunk of a class-M node: its smaller neighbours
    int64_t *block_deg;      // [kNumClasses][prep grid]
    int64_t *units;          // [kNumUnits][grid] work counters per round workgroup
    Counters *ct;
    Barrier *bar;
    int32_t *trace;          // |WL_r| per round
    int64_t *trace_deg;      // degree sum over WL_r per round
    int64_t trace_cap;
    uint64_t *ticks;         // optional timeline: wall clock at each step start
    int64_t tick_cap;
    int64_t threshold;       // topology round iff |WL| > threshold
    int64_t m;
    int32_t n;
    int32_t light_max;
    int32_t hub_min;         // degree above which a node is class M
    int32_t sorted;          // every row strictly ascending
    int32_t grid;            // workgroups of the round kernels (segments per class)
    int32_t light_pull;      // kPushAll, kPullLight or kPullOnly: how class L learns its neighbours' colors
    int32_t racy;            // in-place mode: losers uncolor at once, L assigns avoid in-flight tentatives
    int32_t discard;         // topology-driven rounds keep no worklist; it is rebuilt when data rounds start
    int32_t tail_groups;     // workgroups that stay in the round loop for small data-driven rounds (0: all)
    uint64_t bar_limit;      // wall-clock ticks a grid-barrier wait may last
    const int32_t *gthr;     // a batch with per-graph schedules: H_g per graph (null: one decision per round)
    uint32_t *gsplit;        // per-graph schedules, stepped launches: bit g set iff graph g runs
                             // topology-driven in the current round (the assign launch writes it)
    int32_t *trace_topo;     // per-graph schedules: graphs run topology-driven per round (null: not kept)
    int64_t topo_cap;        // entries of trace_topo
    int32_t ngraphs;         // per-graph schedules: graphs in the batch

    // global id of a neighbour stored in row entry k of node v
    __device__ __forceinline__ int32_t base(int32_t v) const { return gbase ? gbase[v] : 0; }
    // one past the last valid neighbour id of node v (its graph's end)
    __device__ __forceinline__ int64_t id_end(int32_t v) const { return gidx ? gend[gidx[v]] : n; }
    // shift of the byte maps of node v's graph (every neighbour of v shares it)
    __device__ __forceinline__ int64_t fshift(int32_t v) const { return gfshift ? gfshift[gidx[v]] : 0; }
};

// Byte map of node w: bytes [pos, pos + size) for colors 1..size.
struct MapRef {
    uint64_t pos;
    uint32_t size;
};

template <class D>
__device__ __forceinline__ MapRef map_of(const D &d, int32_t w, int64_t fsh) {
    const int64_t a = d.rowptr[w], e = d.rowptr[w + 1];
    return MapRef{(uint64_t)(a + w + fsh), (uint32_t)(e - a) + 1u};
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below() {
    const int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

__device__ __forceinline__ int32_t iabs(int32_t x) { return x < 0 ? -x : x; }

__device__ __forceinline__ int node_class(int64_t d, int light_max, int hub_min) {
    return d <= light_max ? kL : (d <= hub_min ? kW : kM);
}

__device__ __forceinline__ unsigned ld_agent(unsigned *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(unsigned *p, unsigned v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned add_agent(unsigned *p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned xcc_id() {
    // XCC_ID hardware register (id 20), bits [3:0]
    return (unsigned)__builtin_amdgcn_s_getreg(20 | (0 << 6) | (3 << 11)) & (kMaxXcc - 1);
}

// ============================================================== grid barrier

struct GridBarrier {
    Barrier *b;
    unsigned xcc, nxcc, gen;
    unsigned xs;      // participating workgroups on this workgroup's XCD
    uint64_t limit;   // wall-clock ticks any one wait may last

    // True once this wait should end without the barrier: it has lasted longer
    // than the limit (then every other workgroup is told to leave too), or
    // another workgroup gave up.
    __device__ __forceinline__ bool give_up(uint64_t t0) const {
        if (ld_agent(&b->abort.v)) return true;
        if (wall_clock64() - t0 > limit) {
            st_agent(&b->abort.v, 1u);
            return true;
        }
        return false;
    }

    // One-time setup: count the workgroups of every XCD (flat barrier with a
    // per-workgroup release and acquire; used once per launch).  False if the
    // wait gave up: the caller leaves the kernel.
    __device__ __forceinline__ bool setup(Barrier *bar, uint64_t lim) {
        __shared__ int s_ok;
        b = bar;
        limit = lim;
        xcc = xcc_id();
        if (threadIdx.x == 0) {
            add_agent(&b->xsize[xcc].v, 1u);
            b->xcc_of[blockIdx.x] = xcc;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            add_agent(&b->setup.v, 1u);
            const uint64_t t0 = wall_clock64();
            int ok = 1;
            while (ld_agent(&b->setup.v) < gridDim.x) {
                if (give_up(t0)) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok;
        }
        __syncthreads();
        nxcc = 0;
        for (int i = 0; i < kMaxXcc; ++i) nxcc += ld_agent(&b->xsize[i].v) > 0;
        xs = ld_agent(&b->xsize[xcc].v);
        gen = 0;
        return s_ok != 0;
    }

    // From now on only workgroups 0 .. g-1 take part (every one of them calls
    // this at the same point, between two barriers; the others have left).
    __device__ __forceinline__ void shrink(int g) {
        __shared__ unsigned s_x[kMaxXcc];
        if (threadIdx.x < kMaxXcc) s_x[threadIdx.x] = 0;
        __syncthreads();
        for (int i = threadIdx.x; i < g; i += blockDim.x) atomicAdd(&s_x[b->xcc_of[i] & (kMaxXcc - 1)], 1u);
        __syncthreads();
        xs = s_x[xcc];
        nxcc = 0;
        for (int i = 0; i < kMaxXcc; ++i) nxcc += s_x[i] > 0;
        __syncthreads();
    }

    // False if the wait gave up (the caller leaves the kernel).  A leader that
    // gives up does not release its XCD, so no workgroup goes on past a barrier
    // that not every workgroup reached.
    __device__ __forceinline__ bool sync() {
        __shared__ int s_ok;
        __builtin_amdgcn_s_waitcnt(0);  // this thread's stores have reached the XCD's L2
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned g = gen;
            const uint64_t t0 = wall_clock64();
            int ok = 1;
            if (add_agent(&b->xcnt[xcc].v, 1u) == xs - 1) {
                st_agent(&b->xcnt[xcc].v, 0u);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write back this XCD's L2
                if (add_agent(&b->gcnt.v, 1u) == nxcc - 1) {
                    st_agent(&b->gcnt.v, 0u);
                    st_agent(&b->gen.v, g + 1);
                } else {
                    while (ld_agent(&b->gen.v) == g) {
                        if (give_up(t0)) {
                            ok = 0;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                if (ok) st_agent(&b->xgen[xcc].v, g + 1);
            } else {
                while (ld_agent(&b->xgen[xcc].v) == g) {
                    if (give_up(t0)) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            s_ok = ok;
        }
        gen += 1;
        __syncthreads();
        // every thread reads s_ok before it arrives at the next sync, whose write of s_ok
        // follows that sync's first workgroup barrier
        return s_ok != 0;
    }
};

// Zero fill of bytes [p, p + bytes): single bytes up to the first 16-byte
// boundary, 16-byte stores, then the tail.  Used instead of hipMemsetAsync
// for counters, barriers and scratch memory.
static __global__ __launch_bounds__(256) void k_zero(unsigned char *p, uint64_t bytes) {
    const uint64_t gt = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t head = std::min<uint64_t>(bytes, (16 - ((uintptr_t)p & 15)) & 15);
    const uint64_t n16 = (bytes - head) / 16;
    if (gt < head) p[gt] = 0;
    uint4 *q = reinterpret_cast<uint4 *>(p + head);
    for (uint64_t i = gt; i < n16; i += nt) q[i] = make_uint4(0u, 0u, 0u, 0u);
    for (uint64_t i = head + 16 * n16 + gt; i < bytes; i += nt) p[i] = 0;
}

// ============================================================== preparation

// Block-wide exclusive scan of one int per thread (any block size <= 1024).
__device__ __forceinline__ int block_scan(int x, int *total) {
    __shared__ int s_wave[32];
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    int incl = x;
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o);
        if (lane >= o) incl += y;
    }
    if (lane == kWave - 1) s_wave[w] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < nw; ++i) {
            const int t = s_wave[i];
            s_wave[i] = acc;
            acc += t;
        }
        s_wave[31] = acc;
    }
    __syncthreads();
    const int excl = s_wave[w] + incl - x;
    *total = s_wave[31];
    __syncthreads();
    return excl;
}

// Three block-wide exclusive scans at once (one int per thread each), with
// the barriers of one.
__device__ __forceinline__ void block_scan3(const int (&x)[3], int (&ex)[3], int (&total)[3]) {
    __shared__ int s_wave[3][32];
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = (blockDim.x + kWave - 1) / kWave;
    int incl[3] = {x[0], x[1], x[2]};
    for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int y = __shfl_up(incl[k], o);
            if (lane >= o) incl[k] += y;
        }
    }
    if (lane == kWave - 1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) s_wave[k][w] = incl[k];
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        int acc = 0;
        for (int i = 0; i < nw; ++i) {
            const int t = s_wave[threadIdx.x][i];
            s_wave[threadIdx.x][i] = acc;
            acc += t;
        }
        s_wave[threadIdx.x][31] = acc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ex[k] = s_wave[k][w] + incl[k] - x[k];
        total[k] = s_wave[k][31];
    }
    __syncthreads();
}

// Ordered append of the flagged threads of the workgroup: returns each flagged
// thread's position after *count and advances *count (shared) by the total.
__device__ __forceinline__ int block_append(bool flag, int *count) {
    int tot;
    const int ex = block_scan(flag ? 1 : 0, &tot);
    const int base = *count;
    __syncthreads();
    if (threadIdx.x == 0) *count = base + tot;
    __syncthreads();
    return base + ex;
}

// Initial state (Section II-C: every node starts uncolored, every node is in
// the worklist), classes, byte-map metadata, row-pointer checks, and the class
// counts of each workgroup's node range.  Workgroup b covers nodes
// [b*span, (b+1)*span).
//
// With `check`, the rows of class L are checked here too (ids inside the node's
// graph, strictly ascending), four entries at a time; a row is read only if its
// own bounds are valid.  Rows of classes W and M are checked while their rings
// are built.
template <class D>
__global__ __launch_bounds__(kPrepBlock) void k_init(D d, int8_t *cls, int32_t span, int32_t check) {
    const int64_t lo = (int64_t)blockIdx.x * span, hi = std::min<int64_t>(lo + span, d.n);
    int cnt[kNumClasses] = {0, 0, 0};
    int64_t deg[kNumClasses] = {0, 0, 0};
    int chunks = 0;  // row chunks of class-M nodes (their rings are built a chunk per wavefront)
    int bad = 0, bad_id = 0, unsorted = 0;
    for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
        // Round 1 assigns color 1 to every node (no neighbour is committed yet), so the state
        // starts there: tentative color 1, and round 1 skips its assign step.
        d.c[v] = -1;
        const int64_t a = d.rowptr[v], e = d.rowptr[v + 1];
        const bool b = a < 0 || e < a || e > d.m || e - a >= INT32_MAX;
        bad |= b;
        const int64_t dv = b ? 0 : e - a;
        const int k = node_class(dv, d.light_max, d.hub_min);
        cls[v] = (int8_t)k;
        cnt[k] += 1;
        deg[k] += dv;
        if (k == kM) chunks += (int)((dv + kRingChunk - 1) / kRingChunk);
        if (check && k == kL && dv > 0) {
            const int64_t glo = d.base((int32_t)v), ghi = d.id_end((int32_t)v);
            int64_t prev = -1;
            for (int64_t k0 = a; k0 < e; k0 += 4) {
                int64_t u[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) u[j] = k0 + j < e ? (int64_t)d.colidx[k0 + j] + glo : INT64_MAX;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (k0 + j >= e) continue;
                    bad_id |= (u[j] < glo || u[j] >= ghi);
                    unsorted |= (u[j] <= prev);
                    prev = u[j];
                }
            }
        }
    }
    if (__ballot(bad) && lane_id() == 0) d.ct->bad_rows = 1;
    if (__ballot(bad_id) && lane_id() == 0) d.ct->bad_ids = 1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {  // the CSR ends: rowptr[0] == 0 and rowptr[n] == m
        const int64_t r0 = d.rowptr[0], rn = d.rowptr[d.n];
        d.ct->ends[0] = r0;
        d.ct->ends[1] = rn;
        if (r0 != 0 || rn != d.m) d.ct->bad_ends = 1;
    }
    if (__ballot(unsorted) && lane_id() == 0) d.ct->unsorted = 1;
    __shared__ int s_cnt[kNumClasses + 1];
    __shared__ unsigned long long s_deg[kNumClasses];
    if (threadIdx.x <= kNumClasses) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x < kNumClasses) s_deg[threadIdx.x] = 0;
    __syncthreads();
    for (int k = 0; k < kNumClasses; ++k) {
        const int64_t ds = wave_sum(deg[k]);
        const int64_t cs = wave_sum(cnt[k]);
        if (lane_id() == 0) {
            atomicAdd(&s_cnt[k], (int)cs);
            atomicAdd(&s_deg[k], (unsigned long long)ds);
        }
    }
    const int64_t hs = wave_sum(chunks);
    if (lane_id() == 0 && hs) atomicAdd(&s_cnt[kNumClasses], (int)hs);
    __syncthreads();
    if (threadIdx.x <= kNumClasses) d.block_cnt[threadIdx.x * gridDim.x + blockIdx.x] = s_cnt[threadIdx.x];
    if (threadIdx.x < kNumClasses) d.block_deg[threadIdx.x * gridDim.x + blockIdx.x] = (int64_t)s_deg[threadIdx.x];
}

// Prefix of the per-workgroup class counts (one workgroup): static-list
// offsets per preparation workgroup, class sizes and regions, segment sizes,
// and the offsets of each workgroup's first class-M row chunk.  Thread t sums
// the counts of workgroups [t*per, (t+1)*per) (independent loads), one
// workgroup scan combines the sums, and thread t writes its range's offsets.
template <class D>
__global__ __launch_bounds__(1024) void k_offsets(D d, int32_t prep_grid) {
    const int32_t per = (prep_grid + (int32_t)blockDim.x - 1) / (int32_t)blockDim.x;
    const int32_t b0 = min<int32_t>(prep_grid, (int32_t)threadIdx.x * per), b1 = min<int32_t>(prep_grid, b0 + per);
    __shared__ unsigned long long s_d;
    int32_t base = 0;
    for (int k = 0; k <= kNumClasses; ++k) {  // the classes, then the class-M row chunks
        int32_t *row = d.block_cnt + (int64_t)k * prep_grid;
        int32_t sum = 0;
        int64_t ds = 0;
#pragma unroll 8
        for (int32_t b = b0; b < b1; ++b) {  // unrolled: eight loads in flight, not one
            sum += row[b];
            if (k < kNumClasses) ds += d.block_deg[(int64_t)k * prep_grid + b];
        }
        int tot;
        const int ex = block_scan(sum, &tot);
        int32_t acc = (k < kNumClasses ? base : 0) + ex;
#pragma unroll 8
        for (int32_t b = b0; b < b1; ++b) {
            const int32_t x = row[b];
            row[b] = acc;
            acc += x;
        }
        if (k == kNumClasses) {
            if (threadIdx.x == 0) d.ct->hub_chunks = tot;
            break;
        }
        base += tot;
        if (threadIdx.x == 0) s_d = 0;
        __syncthreads();
        const int64_t wsum = wave_sum(ds);
        if (lane_id() == 0 && wsum) atomicAdd(&s_d, (unsigned long long)wsum);
        __syncthreads();
        if (threadIdx.x == 0) d.ct->class_deg[k] = (int64_t)s_d;
        __syncthreads();
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        // block_cnt now holds exclusive offsets; class boundaries from workgroup 0's offsets
        int32_t off[kNumClasses + 1];
        off[0] = 0;
        for (int k = 1; k < kNumClasses; ++k) off[k] = d.block_cnt[k * prep_grid];
        off[kNumClasses] = d.n;
        int64_t so = 0;
        for (int k = 0; k < kNumClasses; ++k) {
            d.ct->static_off[k] = off[k];
            d.ct->class_n[k] = off[k + 1] - off[k];
            // a round of both kinds (per-graph schedules) appends the losers of two passes
            const int32_t cap = ((d.ct->class_n[k] + d.grid - 1) / d.grid + kRoundBlock) * (d.gthr ? 2 : 1);
            d.ct->seg_cap[k] = cap;
            d.ct->seg_off[k] = so;
            so += (int64_t)cap * d.grid;
        }
        d.ct->static_off[kNumClasses] = d.n;
        d.ct->seg_off[kNumClasses] = so;
        d.ct->static_ident = d.n > 0 && (d.ct->class_n[kL] == d.n || d.ct->class_n[kW] == d.n);
        if (d.hub_pre) d.hub_pre[d.ct->class_n[kM]] = d.ct->hub_chunks;
    }
}

// The static list: every node grouped by class, ascending id within a class.
// For class-M nodes also the first of their row chunks (hub_pre, in the same
// order), for k_prep_hubs.
//
// Also the state that only pushes use (light_mode 0: pushes forced; or any node
// of class W/M, which receive pushes): empty color masks and, for class L, every
// row position pending.
template <class D>
__global__ __launch_bounds__(kPrepBlock) void k_fill_static(D d, int32_t span, int32_t light_mode) {
    const int64_t lo = (int64_t)blockIdx.x * span, hi = std::min<int64_t>(lo + span, d.n);
    if (light_mode == 0 || d.ct->class_n[kW] + d.ct->class_n[kM] > 0) {
        for (int64_t v = lo + threadIdx.x; v < hi; v += blockDim.x) {
            d.mask[v] = 0;
            const int64_t dv = d.rowptr[v + 1] - d.rowptr[v];  // checked by k_init before any use
            d.pend[v] = d.cls[v] != kL ? 0u : dv >= 32 ? ~0u : (1u << dv) - 1u;
        }
    }
    if (d.ct->static_ident) return;
    int32_t base[kNumClasses];
    for (int k = 0; k < kNumClasses; ++k) base[k] = d.block_cnt[k * gridDim.x + blockIdx.x];
    int32_t cbase = d.block_cnt[kNumClasses * gridDim.x + blockIdx.x];  // this workgroup's first chunk
    const int32_t m0 = d.ct->static_off[kM];
    const bool hubs = d.hub_pre && d.ct->class_n[kM] > 0;
    for (int64_t v0 = lo; v0 < hi; v0 += blockDim.x) {
        const int64_t v = v0 + threadIdx.x;
        const int k = v < hi ? d.cls[v] : -1;
        for (int q = 0; q < kNumClasses; ++q) {
            int tot;
            const int ex = block_scan(k == q, &tot);
            if (k == q) d.static_list[base[q] + ex] = (int32_t)v;
            if (q == kM && hubs) {
                int ch = 0;
                if (k == kM) ch = (int)((d.rowptr[v + 1] - d.rowptr[v] + kRingChunk - 1) / kRingChunk);
                int ctot;
                const int cex = block_scan(ch, &ctot);
                if (k == kM) d.hub_pre[base[kM] - m0 + ex] = cbase + cex;
                cbase += ctot;
            }
            base[q] += tot;
        }
    }
}

// Ring building reads P chunks of 64 row entries per step, so that P loads are
// in flight together.
constexpr int kRingPass = 4;

// Row entries k0 + j * 64 + lane (j < P) below k1, of node v whose row ends at
// e: u[j] the entry's id, sel[j] whether it is a smaller neighbour (a ring
// entry).  With check, ids outside [lo, hi) set bad (such an id is never
// selected) and an entry not above its predecessor sets unsorted.
template <int P, class D>
__device__ __forceinline__ void ring_select(const D &d, int32_t v, int64_t k0, int64_t k1, int64_t e, int64_t lo,
                                            int64_t hi, bool (&sel)[P], int32_t (&u)[P], int &bad, int &unsorted,
                                            bool check) {
    const int lane = lane_id();
    int64_t ug[P], nx[P];
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int64_t k = k0 + j * kWave + lane;
        ug[j] = k < k1 ? (int64_t)d.colidx[k] + lo : -1;
        nx[j] = check && k < k1 && k + 1 < e ? (int64_t)d.colidx[k + 1] + lo : INT64_MAX;
    }
#pragma unroll
    for (int j = 0; j < P; ++j) {
        const int64_t k = k0 + j * kWave + lane;
        const bool ok = ug[j] >= lo && ug[j] < hi;
        if (check && k < k1) {
            bad |= !ok;
            unsorted |= nx[j] <= ug[j];
        }
        u[j] = (int32_t)ug[j];
        sel[j] = ok && u[j] < v;
    }
}

// Ring of W/M node v, built by one wavefront in one pass over its row, which
// it also checks (ids inside [lo, hi), strictly ascending): the node's smaller
// neighbours in row order, from position 0 of its region [0, d).  (Putting the
// neighbours of class W/M first, which stay uncolored longest, made the rounds
// no faster and cost a class lookup per entry.)
template <class D>
__device__ void ring_build_wave(const D &d, int32_t v, int64_t lo, int64_t hi, int &bad, int &unsorted) {
    const int64_t b = d.rowptr[v], e = d.rowptr[v + 1];
    int32_t nl = 0;  // smaller neighbours written so far
    constexpr int P = kRingPass;
    for (int64_t k0 = b; k0 < e; k0 += P * kWave) {
        bool sel[P];
        int32_t u[P];
        ring_select<P>(d, v, k0, e, e, lo, hi, sel, u, bad, unsorted, true);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint64_t m = __ballot(sel[j]);
            if (sel[j]) d.lower[b + nl + __popcll(m & lanes_below())] = u[j];
            nl += __popcll(m);
        }
    }
    if (lane_id() == 0) {
        d.lstart[v] = 0;
        d.llen[v] = nl;
    }
}

// The same ring and checks for four W nodes at once, a quarter wavefront (16 lanes) each, for rows
// of at most 1024 entries, where a wavefront per node would leave most of its lanes idle.  The
// pass loop runs for the longest of the four rows; has: this quarter holds a node.
template <class D>
__device__ __forceinline__ void ring_build_quarter(const D &d, int32_t v, bool has, int &bad, int &unsorted) {
    constexpr int Q = 16, P = kRingPass;
    const int lane = lane_id(), grp = lane / Q, gl = lane % Q;
    int64_t b = 0, e = 0, lo = 0, hi = 0;
    if (has) {
        b = d.rowptr[v];
        e = d.rowptr[v + 1];
        lo = d.base(v);
        hi = d.id_end(v);
    }
    int64_t len = e - b;
    len = max(len, (int64_t)__shfl_xor((long long)len, 16));
    len = max(len, (int64_t)__shfl_xor((long long)len, 32));
    const uint64_t mine = 0xFFFFull << (grp * Q), below = ((1ull << gl) - 1) << (grp * Q);
    int32_t nl = 0;
    for (int64_t k0 = 0; k0 < len; k0 += P * Q) {
        int64_t ug[P], nx[P];
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int64_t k = b + k0 + j * Q + gl;
            ug[j] = k < e ? (int64_t)d.colidx[k] + lo : -1;
            nx[j] = k + 1 < e ? (int64_t)d.colidx[k + 1] + lo : INT64_MAX;
        }
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const int64_t k = b + k0 + j * Q + gl;
            const bool ok = ug[j] >= lo && ug[j] < hi;
            if (k < e) {
                bad |= !ok;
                unsorted |= nx[j] <= ug[j];
            }
            const bool sel = ok && (int32_t)ug[j] < v;
            const uint64_t m = __ballot(sel) & mine;
            if (sel) d.lower[b + nl + __popcll(m & below)] = (int32_t)ug[j];
            nl += __popcll(m);
        }
    }
    if (has && gl == 0) {
        d.lstart[v] = 0;
        d.llen[v] = nl;
    }
}

// Node at position i of class k's static list (0, 1, ..., n-1 when one class
// holds every node and the list is not written).
template <class D>
__device__ __forceinline__ int32_t static_at(const D &d, int k, int64_t i) {
    const int64_t p = d.ct->static_off[k] + i;
    return d.ct->static_ident ? (int32_t)p : d.static_list[p];
}

// Rings of the class-W nodes (a wavefront each; with hub_pre unset, of the
// class-M nodes too), with the checks of their rows.
template <class D>
__global__ __launch_bounds__(kPrepBlock) void k_prep_wide(D d) {
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    const int32_t nWide = d.ct->class_n[kW] + (d.hub_pre ? 0 : d.ct->class_n[kM]);
    int bad = 0, unsorted = 0;
    if (d.hub_pre && d.hub_min <= 1024) {  // only class W here, rows of at most 1024 entries
        const int grp = lane_id() / 16;
        for (int64_t i0 = gw * 4; i0 < nWide; i0 += nw * 4) {  // the same for the whole wavefront
            const int64_t i = i0 + grp;
            const bool has = i < nWide;
            ring_build_quarter(d, has ? static_at(d, kW, i) : 0, has, bad, unsorted);
        }
    } else {
        for (int64_t i = gw; i < nWide; i += nw) {
            const int32_t v = static_at(d, kW, i);
            ring_build_wave(d, v, d.base(v), d.id_end(v), bad, unsorted);
        }
    }
    if (__ballot(bad) && lane_id() == 0) d.ct->bad_ids = 1;
    if (__ballot(unsorted) && lane_id() == 0) d.ct->unsorted = 1;
}

// Part of class-M node v's ring from row entries [k0, k1) of its row [b, e),
// by one wavefront.  Counting pass (WRITE false): the chunk's smaller
// neighbours (returned), with the checks of its entries.  Placing pass: the same
// neighbours, in row order, at ring positions pos.., so that the ring is laid
// out exactly as ring_build_wave lays it out.
template <bool WRITE, class D>
__device__ int32_t ring_build_chunk(const D &d, int32_t v, int64_t b, int64_t e, int64_t k0, int64_t k1, int64_t lo,
                                    int64_t hi, int32_t pos, int &bad, int &unsorted) {
    int32_t nl = 0;
    constexpr int P = kRingPass;
    for (int64_t p = k0; p < k1; p += P * kWave) {
        bool sel[P];
        int32_t u[P];
        ring_select<P>(d, v, p, k1, e, lo, hi, sel, u, bad, unsorted, !WRITE);
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const uint64_t m = __ballot(sel[j]);
            if (WRITE && sel[j]) d.lower[b + pos + nl + __popcll(m & lanes_below())] = u[j];
            nl += __popcll(m);
        }
    }
    return nl;
}

// Rings of the class-M nodes: their rows are cut into chunks of kRingChunk
// entries (hub_pre: first chunk of each node, in static-list order), and
// wavefront w of the grid takes chunks w, w + waves, ...; a node of degree 10^5
// costs about as much as fifty of degree 2048 instead of one wavefront walking
// its whole row.  Two launches: WRITE false counts each chunk's smaller
// neighbours into hub_cnt and checks the entries; WRITE true places them from
// the prefix of the node's chunk counts and sets the ring's start and length.
template <bool WRITE, class D>
__global__ __launch_bounds__(kPrepBlock) void k_prep_hubs(D d) {
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    const int32_t nM = d.ct->class_n[kM];
    const int32_t total = d.hub_pre[nM];
    int bad = 0, unsorted = 0;
    for (int64_t g = gw; g < total; g += nw) {
        // the node h with hub_pre[h] <= g < hub_pre[h + 1], by a 64-way search (every node has a chunk)
        int64_t lo = 0, hi = nM;
        while (hi - lo > 1) {
            const int64_t step = (hi - lo + kWave - 1) / kWave;
            const int64_t idx = lo + lane * step;
            const uint64_t le = __ballot(idx < hi && d.hub_pre[idx] <= g);
            lo += (int64_t)(63 - __clzll((unsigned long long)le)) * step;
            hi = min(hi, lo + step);
        }
        const int32_t v = static_at(d, kM, lo);
        const int64_t b = d.rowptr[v], e = d.rowptr[v + 1];
        const int32_t c0 = d.hub_pre[lo], c1 = d.hub_pre[lo + 1];
        const int64_t k0 = b + (g - c0) * (int64_t)kRingChunk, k1 = min<int64_t>(k0 + kRingChunk, e);
        if (!WRITE) {
            const int32_t nl = ring_build_chunk<false>(d, v, b, e, k0, k1, d.base(v), d.id_end(v), 0, bad, unsorted);
            if (lane == 0) d.hub_cnt[g] = nl;
        } else {
            int64_t before = 0, all = 0;  // this node's chunks before g, and all of them
            for (int64_t c = c0 + lane; c < c1; c += kWave) {
                const int32_t x = d.hub_cnt[c];
                before += c < g ? x : 0;
                all += x;
            }
            before = wave_sum(before);
            all = wave_sum(all);
            ring_build_chunk<true>(d, v, b, e, k0, k1, d.base(v), d.id_end(v), (int32_t)before, bad, unsorted);
            if (g == c0 && lane == 0) {
                d.lstart[v] = 0;
                d.llen[v] = (int32_t)all;
            }
        }
    }
    if (!WRITE) {
        if (__ballot(bad) && lane == 0) d.ct->bad_ids = 1;
        if (__ballot(unsorted) && lane == 0) d.ct->unsorted = 1;
    }
}

// ============================================================== full validation
//
// IPGC_VALIDATE_FULL: the input must be a simple symmetric graph (Section V
// colors graphs with self-loops and multi-edges removed; the method is defined
// on undirected graphs).  k_full_sort writes every row, sorted, into a scratch
// array with the CSR's layout; k_full_check then flags a self-loop, a repeated
// id in a row, or an entry (v, u) with no reverse entry (u, v), found by binary
// search in the sorted row of u.  Every entry's reverse present and no
// repeated entries make the CSR exactly symmetric.

constexpr int kSortBlock = 256;
constexpr int kSortShared = 4096;  // rows up to this length are sorted in shared memory

enum { kFullSelfLoop = 1, kFullDuplicate = 2, kFullAsymmetric = 4 };

// Sorts a[0, len) ascending with the whole workgroup.  A bitonic network in
// which every comparator puts the smaller value at the lower position (the
// first stage of each merge pairs mirrored positions), so positions at or past
// len act as +infinity: a comparator that reaches one would never swap, and is
// skipped.  Stages are separated by workgroup barriers; `a` is shared or
// global memory of this workgroup alone.
__device__ void workgroup_sort(int32_t *a, int64_t len) {
    int64_t N = 1;
    while (N < len) N <<= 1;
    for (int64_t k = 2; k <= N; k <<= 1) {
        for (int64_t j = k - 1; j > 0; j = (j == k - 1) ? (k >> 2) : (j >> 1)) {
            for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
                const int64_t q = i ^ j;
                if (q > i && q < len) {
                    const int32_t x = a[i], y = a[q];
                    if (y < x) {
                        a[i] = y;
                        a[q] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
}

// Every row of nodes [v_lo, v_hi), sorted, into out (same positions as colidx).
// Nothing is read if *skip is set (a server job whose rows failed their checks).
template <class D>
__global__ __launch_bounds__(kSortBlock) void k_full_sort(D d, int64_t v_lo, int64_t v_hi, int32_t *out,
                                                          const int32_t *skip) {
    __shared__ int32_t s[kSortShared];
    if (skip && *skip) return;
    for (int64_t v = v_lo + blockIdx.x; v < v_hi; v += gridDim.x) {
        const int64_t b = d.rowptr[v], len = d.rowptr[v + 1] - b;
        int unsorted = 0;
        for (int64_t i = threadIdx.x; i < len; i += blockDim.x) {
            const int32_t x = d.colidx[b + i];
            out[b + i] = x;
            if (i + 1 < len && d.colidx[b + i + 1] < x) unsorted = 1;
        }
        if (!__syncthreads_or(unsorted)) continue;  // ascending already: the copy stands
        if (len <= kSortShared) {
            for (int64_t i = threadIdx.x; i < len; i += blockDim.x) s[i] = out[b + i];
            __syncthreads();
            workgroup_sort(s, len);
            for (int64_t i = threadIdx.x; i < len; i += blockDim.x) out[b + i] = s[i];
            __syncthreads();
        } else {
            workgroup_sort(out + b, len);
        }
    }
}

// Checks of nodes [v_lo, v_hi) on the sorted rows (a wavefront per node); the
// kFull* bits found are ORed into *flag.  Ids outside the node's graph are left
// to the range checks (and never used as an index here).
template <class D>
__global__ __launch_bounds__(kPrepBlock) void k_full_check(D d, int64_t v_lo, int64_t v_hi, const int32_t *rows,
                                                           int32_t *flag, const int32_t *skip) {
    if (skip && *skip) return;
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    const int lane = lane_id();
    int bad = 0;
    for (int64_t v = v_lo + gw; v < v_hi; v += nw) {
        const int64_t b = d.rowptr[v], e = d.rowptr[v + 1];
        const int64_t lo = d.base((int32_t)v), hi = d.id_end((int32_t)v);
        const int32_t vl = (int32_t)(v - lo);  // v's id inside its graph, as its neighbours' rows hold it
        for (int64_t k = b + lane; k < e; k += kWave) {
            const int32_t ul = rows[k];
            const int64_t u = (int64_t)ul + lo;
            if (u < lo || u >= hi) continue;
            if (u == v) bad |= kFullSelfLoop;
            if (k + 1 < e && rows[k + 1] == ul) bad |= kFullDuplicate;
            int64_t a = d.rowptr[u], z = d.rowptr[u + 1];
            const int64_t end = z;
            while (a < z) {  // first position of row u holding an id >= vl
                const int64_t mid = (a + z) >> 1;
                if (rows[mid] < vl) a = mid + 1;
                else z = mid;
            }
            if (a == end || rows[a] != vl) bad |= kFullAsymmetric;
        }
    }
    for (int o = 32; o > 0; o >>= 1) bad |= __shfl_xor(bad, o);
    if (bad && lane == 0) atomicOr(flag, bad);
}

// A packed batch seen as one graph: union row starts (local offsets of graph
// g shifted by its first entry), the first global id of each node's graph,
// and each node's graph index.  A workgroup per graph at a time; also checks
// each graph's row pointers (local rowptr[0] == 0, rowptr[n_g] == m_g,
// non-decreasing) and flags bad_rows.
static __global__ __launch_bounds__(kPrepBlock) void k_batch_union(const int64_t *node_off, const int64_t *edge_off,
                                                            const int32_t *rowptr_packed, int64_t graphs,
                                                            int64_t *growptr, int32_t *gbase, int32_t *gidx,
                                                            Counters *ct) {
    int bad = 0;
    for (int64_t g = blockIdx.x; g < graphs; g += gridDim.x) {
        const int64_t n0 = node_off[g], ng = node_off[g + 1] - n0;
        const int64_t e0 = edge_off[g], mg = edge_off[g + 1] - e0;
        const int32_t *rp = rowptr_packed + n0 + g;  // graph g's n_g + 1 local row pointers
        for (int64_t lv = threadIdx.x; lv <= ng; lv += blockDim.x) {
            const int64_t a = rp[lv];
            if (lv == 0) bad |= a != 0;
            if (lv == ng) bad |= a != mg;
            if (lv < ng) {
                const int64_t e = rp[lv + 1];
                bad |= e < a || a < 0 || e > mg;
                growptr[n0 + lv] = e0 + a;
                gbase[n0 + lv] = (int32_t)n0;
                gidx[n0 + lv] = (int32_t)g;
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) growptr[node_off[graphs]] = edge_off[graphs];
    if (__ballot(bad) && lane_id() == 0) ct->bad_rows = 1;
}

// ============================================================== worklist views

// The items of one class in the round's input: either the static list (a
// topology-driven sweep, or round 1) or the segmented list of the previous
// round, read through the prefix sums of its segment counts.
struct ClassView {
    const int32_t *base;  // static: first entry of the class (null: the list 0, 1, ..., n-1); segmented:
                          // first segment of the class
    const int32_t *pre;   // segmented: shared-memory prefix sums (grid + 1 entries), else null
    int32_t cap;          // segmented: entries per segment
    int32_t total;

    // the segment s in [lo, hi) with pre[s] <= i < pre[s + 1] (pre[lo] <= i is assumed)
    __device__ __forceinline__ int seg_of(int32_t i, int lo, int hi) const {
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pre[mid] <= i) lo = mid;
            else hi = mid;
        }
        return lo;
    }

    // item i, found among segments [lo, hi) (see range)
    __device__ __forceinline__ int32_t at_in(int32_t i, int lo, int hi) const {
        if (!pre) return base ? base[i] : i;  // null base: the static list 0, 1, ..., n-1
        const int s = seg_of(i, lo, hi);
        return base[(int64_t)s * cap + (i - pre[s])];
    }

    __device__ __forceinline__ int32_t at(int32_t i) const { return at_in(i, 0, gridDim.x); }

    // Segments [*lo, *hi) holding items a..b (a <= b < total; the same for every lane of a
    // wavefront), so that each lane's search for an item in between covers only those: in large
    // rounds a wavefront's items lie in one or two segments.
    __device__ __forceinline__ void range(int32_t a, int32_t b, int *lo, int *hi) const {
        if (!pre) {
            *lo = 0;
            *hi = 1;
            return;
        }
        *lo = seg_of(a, 0, gridDim.x);
        *hi = seg_of(b, *lo, gridDim.x) + 1;
    }
};

struct RoundIn {
    ClassView cv[kNumClasses];
    int32_t wl[kNumClasses];  // worklist entries per class (the active nodes)
    int32_t total;            // worklist size |WL_r|
    bool topo;
    bool split;               // per-graph schedules, a round of both kinds: this view takes only the nodes
                              // of graphs whose kind of round is `topo` (graph_bits)
};

// ============================================================== per-graph schedules (batches)
//
// With per-graph thresholds every graph of a batch takes the decision of Section IV on its own:
// its round r is topology-driven iff its worklist (its nodes not yet committed, gleft) holds more
// than H_g nodes.  A round in which graphs of both kinds still have active nodes runs each step
// twice: over the worklist for the nodes of data-driven graphs and as a sweep of the static list
// for the nodes of topology-driven ones.  One graph's nodes are all handled by one of the two
// passes, so every graph sees exactly the round it would see alone.

// The instantiation for batches with per-graph schedules; the others carry none of their code.
template <class D>
constexpr bool kSplitDev = D::kSplit;

// Bit g set iff graph g runs topology-driven in this round (shared memory, one copy per workgroup).
__device__ __forceinline__ uint32_t *graph_bits() {
    __shared__ uint32_t s_bits[kMaxSplitGraphs / 32];
    return s_bits;
}

struct Split {
    int32_t topo;  // graphs with active nodes that run this round topology-driven
    int32_t data;  // graphs with active nodes that run it data-driven
};

// The kind of round of every graph into graph_bits, and how many graphs have each kind.  All
// threads of the workgroup call this while gleft does not change (before any commit of the
// round).  initial: from the node counts, as at the start of round 1.
template <class D>
__device__ __forceinline__ Split graph_split(const D &d, bool initial) {
    __shared__ int s_n[2];
    uint32_t *bits = graph_bits();
    if (threadIdx.x < 2) s_n[threadIdx.x] = 0;
    __syncthreads();
    const int lane = lane_id();
    for (int g0 = (int)(threadIdx.x / kWave) * kWave; g0 < d.ngraphs; g0 += (int)blockDim.x) {
        const int g = g0 + lane;
        int64_t left = 0;
        if (g < d.ngraphs)
            left = initial ? d.gend[g] - (g > 0 ? d.gend[g - 1] : 0) : (int32_t)ld_agent((unsigned *)&d.gleft[g]);
        const bool topo = g < d.ngraphs && left > 0 && left > (int64_t)d.gthr[g];  // a done graph has no round
        const uint64_t tm = __ballot(topo), dm = __ballot(left > 0 && !topo);
        if (lane == 0) {  // kMaxSplitGraphs / 32 words hold 64 graphs per wavefront step
            bits[g0 >> 5] = (uint32_t)tm;
            bits[(g0 >> 5) + 1] = (uint32_t)(tm >> 32);
            if (tm) atomicAdd(&s_n[0], (int)__popcll(tm));
            if (dm) atomicAdd(&s_n[1], (int)__popcll(dm));
        }
    }
    __syncthreads();
    const Split sp{s_n[0], s_n[1]};
    __syncthreads();  // s_n is reset by the next call
    return sp;
}

// True if item v of a view is not this view's work: a committed node met by a sweep, or, in a
// round of both kinds, a node of a graph handled by the other pass.
template <class D>
__device__ __forceinline__ bool skip_item(const D &d, const RoundIn &in, int32_t v, int32_t cv) {
    bool skip = in.topo && cv > 0;
    if constexpr (kSplitDev<D>) {
        if (in.split) {
            const int32_t g = d.gidx[v];
            skip = skip || (bool)(graph_bits()[g >> 5] >> (g & 31) & 1u) != in.topo;
        }
    }
    return skip;
}

// Load the segment counts of list `src` and build the prefix sums in shared
// memory (all threads of the workgroup call this).
// Segments past the first `writers` (workgroups that had left the round loop
// when the list was written) count as empty.
template <class D>
__device__ __forceinline__ void load_segments(const D &d, int src, int32_t (*pre)[kMaxRoundBlocks + 1], int writers) {
    static_assert(kNumClasses == 3, "one fused scan covers the three classes");
    const int nb = gridDim.x;
    int x[kNumClasses], ex[kNumClasses], tot[kNumClasses];
    for (int k = 0; k < kNumClasses; ++k) x[k] = threadIdx.x < (unsigned)writers ? d.seg_cnt[src][k * nb + threadIdx.x] : 0;
    block_scan3(x, ex, tot);
    for (int k = 0; k < kNumClasses; ++k) {
        if (threadIdx.x < (unsigned)nb) pre[k][threadIdx.x] = ex[k];
        if (threadIdx.x == 0) pre[k][nb] = tot[k];
    }
    __syncthreads();
}

// The items of round r: the static list (round 1, topology-driven rounds) or the segmented list.
// force: -1 decides by |WL| > H, 0 and 1 set data- or topology-driven (per-graph schedules).
template <class D>
__device__ __forceinline__ RoundIn round_view(const D &d, int r, int32_t (*pre)[kMaxRoundBlocks + 1], int force = -1) {
    RoundIn in;
    int32_t tot[kNumClasses];
    if (r == 1) {
        for (int k = 0; k < kNumClasses; ++k) tot[k] = d.ct->class_n[k];
    } else {
        for (int k = 0; k < kNumClasses; ++k) tot[k] = pre[k][gridDim.x];
    }
    in.total = tot[0] + tot[1] + tot[2];
    for (int k = 0; k < kNumClasses; ++k) in.wl[k] = tot[k];
    in.topo = force < 0 ? (int64_t)in.total > d.threshold : force > 0;
    in.split = false;
    const int src = r & 1;  // round r reads list (r & 1) written by round r-1
    for (int k = 0; k < kNumClasses; ++k) {
        if (r == 1 || in.topo) {
            in.cv[k].base = d.ct->static_ident ? nullptr : d.static_list + d.ct->static_off[k];
            in.cv[k].pre = nullptr;
            in.cv[k].cap = 0;
            in.cv[k].total = d.ct->class_n[k];
        } else {
            in.cv[k].base = d.seg_list[src] + d.ct->seg_off[k];
            in.cv[k].pre = pre[k];
            in.cv[k].cap = d.ct->seg_cap[k];
            in.cv[k].total = tot[k];
        }
    }
    return in;
}

// This workgroup's work-counter totals (shared memory, one set per kernel).
__device__ __forceinline__ unsigned long long *unit_totals() {
    __shared__ unsigned long long s_u[kNumUnits];
    return s_u;
}

// Work counters: 32 bits per thread within a step (a thread counts far fewer
// than 2^32 units in one step of any graph that fits in memory), folded into
// the workgroup's 64-bit shared totals at the end of each step, written to
// d.units[i][block] at the end of the kernel.
struct Units {
    uint32_t u[kNumUnits];
    __device__ __forceinline__ Units() {
        for (int i = 0; i < kNumUnits; ++i) u[i] = 0;
        if (threadIdx.x < kNumUnits) unit_totals()[threadIdx.x] = 0;
        __syncthreads();
    }
    // every thread of the workgroup calls this at the same point
    __device__ __forceinline__ void fold() {
        unsigned long long *tot = unit_totals();
        for (int i = 0; i < kNumUnits; ++i) {
            const int64_t s = wave_sum((int64_t)u[i]);
            if (lane_id() == 0 && s) atomicAdd(&tot[i], (unsigned long long)s);
            u[i] = 0;
        }
    }
    template <class D>
    __device__ __forceinline__ void flush(const D &d) {
        fold();
        __syncthreads();
        if (threadIdx.x < kNumUnits) d.units[threadIdx.x * gridDim.x + blockIdx.x] += (int64_t)unit_totals()[threadIdx.x];
        __syncthreads();
    }
};

// Appends of one workgroup's losers into its own segments of the out list.
struct OutSegs {
    int32_t *list;     // out list
    int32_t *cnt;      // its segment counts
    int64_t *deg;
    int64_t cls_off[kNumClasses];
    int cap[kNumClasses];
};

// ============================================================== step 1: tentative first-fit colors
//
// Every uncolored node takes the smallest color >= 1 that no committed
// neighbour holds (Section II-C with its footnote on mex; 0 marks uncolored).

// First free color of W/M node v from color 65 on (its 64 mask bits are all
// set), a wavefront over its byte map; writes the tentative color.
template <class D>
__device__ __forceinline__ void map_assign_wave(const D &d, int32_t v, Units &un) {
    const int lane = lane_id();
    const int32_t cv = d.c[v];
    const MapRef fm = map_of(d, v, d.fshift(v));
    // from the previous tentative color (0-based; first-fit colors only grow) or color 65
    uint32_t st = max(cv < 0 ? (uint32_t)(-cv) - 1u : 0u, (uint32_t)kMaskColors);
    int32_t t = (int32_t)fm.size;  // d + 1 is free if nothing smaller is
    for (; st < fm.size; st += kWave) {
        const uint32_t idx = st + lane;
        const uint8_t used = idx < fm.size ? d.F[fm.pos + idx] : 0;
        const uint64_t fz = __ballot(used == 0);
        un.u[kUMapBytes] += lane == 0 ? kWave : 0;
        if (fz) {
            t = (int32_t)(st + __ffsll((unsigned long long)fz));
            break;
        }
    }
    if (lane == 0) {
        d.c[v] = -t;
        un.u[kUAssignNodes] += 1;
    }
}

// Class L nodes (degree <= light_max <= 32) run a lane each, kLightK of them in flight per lane:
// each step of the per-node chain (worklist entry, state and row bounds, row entries, neighbour
// states) is issued for all of a lane's nodes before any result is used, so one lane keeps up to
// kLightK * kLightC loads outstanding where a node alone has a chain of dependent ones.  A
// wavefront takes items b0 + j * 64 + lane (j < kLightK) of a block of 64 * kLightK consecutive
// items, so every load of a step is coalesced across the wavefront when the items are.
constexpr int kLightK = 2;  // nodes per lane
constexpr int kLightC = 4;  // row entries per node per pass

// Per-graph schedules, a round of both kinds: the light items of graphs handled by the other
// pass become absent (no node, not active).
template <bool TOPO, class D>
__device__ __forceinline__ void drop_other_part(const D &d, int32_t (&v)[kLightK], uint32_t &act) {
#pragma unroll
    for (int j = 0; j < kLightK; ++j) {
        if (v[j] < 0) continue;
        const int32_t g = d.gidx[v[j]];
        if ((bool)(graph_bits()[g >> 5] >> (g & 31) & 1u) != TOPO) {
            v[j] = -1;
            act &= ~(1u << j);
        }
    }
}

// Tentative colors of the class-L items (Section II-C, first fit): the first zero bit of the
// node's color mask (push modes: committed neighbours set bit t - 1; d <= 32 neighbours leave a
// zero among the first 33 bits), or of a mask of the committed colors read from the
// neighbours' states (pull modes).  TOPO: a sweep over the static list, committed nodes skipped.
// The blocks of a light sweep in a round of both kinds (per-graph schedules): first, first + step,
// ... below total, leaving out blocks that hold only nodes of one data-driven graph.  Each lane
// judges one of the wavefront's next 64 blocks from the graphs of its first and last node (a block
// whose ends lie in different graphs is kept), so 64 blocks cost one round trip.
struct LightBlocks {
    int64_t base, step;
    int32_t total;
    uint64_t keep = 0;  // bit j: block base + j * step still to run
    bool fresh = true;
    __device__ LightBlocks(int64_t first, int64_t step_, int32_t total_) : base(first), step(step_), total(total_) {}
    template <class D>
    __device__ __forceinline__ bool next(const D &d, const ClassView &cv, int64_t *b0) {
        while (!keep) {  // the same for the whole wavefront
            if (!fresh) base += kWave * step;
            fresh = false;
            if (base >= total) return false;
            const int64_t bj = base + (int64_t)lane_id() * step;
            bool k = false;
            if (bj < total) {
                const int32_t v1 = cv.at_in((int32_t)bj, 0, 1);
                const int32_t v2 = cv.at_in((int32_t)min<int64_t>(bj + kWave * kLightK, total) - 1, 0, 1);
                const int32_t g1 = d.gidx[v1], g2 = d.gidx[v2];
                k = g1 != g2 || (graph_bits()[g1 >> 5] >> (g1 & 31) & 1u);
            }
            keep = __ballot(k);
        }
        const int j = __ffsll((unsigned long long)keep) - 1;
        keep &= keep - 1;
        *b0 = base + (int64_t)j * step;
        return true;
    }
};

// The blocks of a light pass: b0 = first, first + step, ... below total.  With per-graph schedules
// compiled in, the sweep of a round of both kinds (filt) leaves out the blocks of data-driven
// graphs; the other instantiations iterate plainly.
template <bool SPLIT>
struct LightIter {
    int64_t step;
    int32_t total;
    __device__ LightIter(int64_t, int64_t step_, int32_t total_, bool) : step(step_), total(total_) {}
    template <class D>
    __device__ __forceinline__ bool more(const D &, const ClassView &, int64_t &b0) const { return b0 < total; }
    __device__ __forceinline__ void advance(int64_t &b0) const { b0 += step; }
};

template <>
struct LightIter<true> {
    LightBlocks lb;
    int64_t step;
    int32_t total;
    bool filt;
    __device__ LightIter(int64_t first, int64_t step_, int32_t total_, bool filt_)
        : lb(first, step_, total_), step(step_), total(total_), filt(filt_) {}
    template <class D>
    __device__ __forceinline__ bool more(const D &d, const ClassView &cv, int64_t &b0) {
        return filt ? lb.next(d, cv, &b0) : b0 < total;
    }
    __device__ __forceinline__ void advance(int64_t &b0) const {
        if (!filt) b0 += step;
    }
};

// Tentative colors of the class-L items (Section II-C, first fit): the first zero bit of the
// node's color mask (push modes: committed neighbours set bit t - 1; d <= 32 neighbours leave a
// zero among the first 33 bits), or of a mask of the committed colors read from the
// neighbours' states (pull modes).  TOPO: a sweep over the static list, committed nodes skipped.
template <bool TOPO, class D>
__device__ __forceinline__ void light_assign(const D &d, const ClassView &cv, bool split, Units &un, int G) {
    using Off = typename D::OffT;
    constexpr int K = kLightK, C = kLightC;
    const int lane = lane_id();
    // blocks of 64 * K items go round the workgroups (block i to workgroup i mod G), so no
    // workgroup takes more than total / G + 64 * K * (1 + 1/G) items: its out segments hold them
    const int64_t gw = (int64_t)(threadIdx.x / kWave) * G + blockIdx.x;
    const int64_t nw = (int64_t)G * (blockDim.x / kWave);
    const int32_t total = cv.total;
    LightIter<kSplitDev<D>> it(gw * (kWave * K), nw * (kWave * K), total, TOPO && split);
    for (int64_t b0 = gw * (kWave * K); it.more(d, cv, b0); it.advance(b0)) {
        int slo, shi;
        cv.range((int32_t)b0, (int32_t)min<int64_t>(b0 + kWave * K, total) - 1, &slo, &shi);
        int32_t v[K];
        uint32_t act = 0;  // bit j: item j of this lane is an active node
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t i = b0 + j * kWave + lane;
            v[j] = i < total ? cv.at_in((int32_t)i, slo, shi) : -1;
            act |= (i < total ? 1u : 0u) << j;
        }
        if constexpr (kSplitDev<D>) {
            if (split) drop_other_part<TOPO>(d, v, act);
        }
        if (TOPO) {
            int32_t c0[K];
    #pragma unroll
            for (int j = 0; j < K; ++j) c0[j] = v[j] >= 0 ? d.c[v[j]] : 1;
    #pragma unroll
            for (int j = 0; j < K; ++j)
                if (c0[j] > 0) act &= ~(1u << j);
        }
        if (d.light_pull == kPushAll) {
            uint64_t mk[K];
    #pragma unroll
            for (int j = 0; j < K; ++j) mk[j] = act >> j & 1u ? d.mask[v[j]] : 0ull;
    #pragma unroll
            for (int j = 0; j < K; ++j)
                if (act >> j & 1u) d.c[v[j]] = -__ffsll((unsigned long long)~mk[j]);
            un.u[kUMapBytes] += 8 * __popc(act);
            un.u[kUAssignNodes] += __popc(act);
            continue;
        }
        Off b[K];
        int32_t len[K], gb[K];
        uint64_t used[K];
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            const bool a = act >> j & 1u;
            b[j] = a ? d.rowptr[v[j]] : 0;
            len[j] = a ? (int32_t)(d.rowptr[v[j] + 1] - b[j]) : 0;
            gb[j] = a ? d.base(v[j]) : 0;
            used[j] = 0;
        }
        for (int32_t q0 = 0;; q0 += C) {
            int32_t cu[K][C];
    #pragma unroll
            for (int j = 0; j < K; ++j)
    #pragma unroll
                for (int q = 0; q < C; ++q) cu[j][q] = q0 + q < len[j] ? d.colidx[b[j] + q0 + q] + gb[j] : -1;
    #pragma unroll
            for (int j = 0; j < K; ++j)
    #pragma unroll
                for (int q = 0; q < C; ++q) cu[j][q] = cu[j][q] >= 0 ? d.c[cu[j][q]] : 0;
            bool more = false;
    #pragma unroll
            for (int j = 0; j < K; ++j) {
    #pragma unroll
                for (int q = 0; q < C; ++q) {
                    const int32_t x = d.racy ? iabs(cu[j][q]) : cu[j][q];  // racy: in-flight tentatives too
                    if (x > 0 && x <= 64) used[j] |= 1ull << (x - 1);
                }
                more |= q0 + C < len[j];
            }
            if (!more) break;
        }
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!(act >> j & 1u)) continue;
            d.c[v[j]] = -__ffsll((unsigned long long)~used[j]);
            un.u[kUPullEntries] += len[j];
        }
        un.u[kUAssignNodes] += __popc(act);
    }
}

// Conflict test, commit and push of the class-L items (Section II-C): v loses iff a smaller
// neighbour holds its tentative color t.  Pull-only graphs scan the row up to v (sorted rows
// stop there); push modes scan only the positions still pending, and drop from them the
// neighbours found committed (their colors have reached v's mask).  Losers go to the
// workgroup's class-L segment with one shared-memory atomic per wavefront (ballot and popcount
// give each its slot); winners commit and, in push modes, set bit t - 1 (t <= 33) in their
// neighbours' masks.
template <bool TOPO, class D>
__device__ __forceinline__ void light_conflict(const D &d, const ClassView &cv, bool split, int64_t seg_base, bool discard,
                                               int32_t r, Units &un, int G, int32_t *list, int32_t seg_cap,
                                               int *s_cnt, unsigned long long *s_deg) {
    using Off = typename D::OffT;
    constexpr int K = kLightK, C = kLightC;
    const int lane = lane_id();
    // blocks of 64 * K items go round the workgroups (block i to workgroup i mod G), so no
    // workgroup takes more than total / G + 64 * K * (1 + 1/G) items: its out segments hold them
    const int64_t gw = (int64_t)(threadIdx.x / kWave) * G + blockIdx.x;
    const int64_t nw = (int64_t)G * (blockDim.x / kWave);
    const int32_t total = cv.total;
    const bool pull_only = d.light_pull == kPullOnly;
    LightIter<kSplitDev<D>> it(gw * (kWave * K), nw * (kWave * K), total, TOPO && split);
    for (int64_t b0 = gw * (kWave * K); it.more(d, cv, b0); it.advance(b0)) {
        int slo, shi;
        cv.range((int32_t)b0, (int32_t)min<int64_t>(b0 + kWave * K, total) - 1, &slo, &shi);
        int32_t v[K], t[K];
        uint32_t act = 0;  // bit j: item j is an active node
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t i = b0 + j * kWave + lane;
            v[j] = i < total ? cv.at_in((int32_t)i, slo, shi) : -1;
            act |= (i < total ? 1u : 0u) << j;
        }
        if constexpr (kSplitDev<D>) {
            if (split) drop_other_part<TOPO>(d, v, act);
        }
    #pragma unroll
        for (int j = 0; j < K; ++j) t[j] = v[j] >= 0 ? -d.c[v[j]] : 0;
        if (TOPO) {
    #pragma unroll
            for (int j = 0; j < K; ++j)
                if (t[j] < 0) act &= ~(1u << j);  // committed (c > 0)
        }
        Off b[K];
        int32_t len[K], gb[K];
        uint32_t pm[K];  // pull-only: unused; push modes: pending positions not yet scanned
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            const bool a = act >> j & 1u;
            b[j] = a ? d.rowptr[v[j]] : 0;
            len[j] = a ? (int32_t)(d.rowptr[v[j] + 1] - b[j]) : 0;
            gb[j] = a ? d.base(v[j]) : 0;
            pm[j] = a && !pull_only ? d.pend[v[j]] : 0u;
        }
        uint32_t lose = 0, done = ~act;  // bit j
        uint32_t seen[K];                // push modes: positions found committed
        int32_t read = 0;
    #pragma unroll
        for (int j = 0; j < K; ++j) seen[j] = 0;
        for (int32_t q0 = 0;; q0 += C) {
            int32_t pos[K][C], u[K][C];
    #pragma unroll
            for (int j = 0; j < K; ++j)
    #pragma unroll
                for (int q = 0; q < C; ++q) {
                    if (pull_only) {
                        pos[j][q] = !(done >> j & 1u) && q0 + q < len[j] ? q0 + q : -1;
                    } else {
                        pos[j][q] = !(done >> j & 1u) && pm[j] ? __ffs(pm[j]) - 1 : -1;
                        pm[j] &= pm[j] - 1;
                    }
                }
    #pragma unroll
            for (int j = 0; j < K; ++j)
    #pragma unroll
                for (int q = 0; q < C; ++q) u[j][q] = pos[j][q] >= 0 ? d.colidx[b[j] + pos[j][q]] + gb[j] : INT32_MAX;
            int32_t cu[K][C];
    #pragma unroll
            for (int j = 0; j < K; ++j)
    #pragma unroll
                for (int q = 0; q < C; ++q) cu[j][q] = u[j][q] < v[j] ? d.c[u[j][q]] : 0;
    #pragma unroll
            for (int j = 0; j < K; ++j) {
    #pragma unroll
                for (int q = 0; q < C; ++q) {
                    if (done >> j & 1u) continue;
                    if (u[j][q] >= v[j]) {  // not a smaller neighbour; past the row's end if INT32_MAX
                        if (d.sorted || u[j][q] == INT32_MAX) done |= 1u << j;
                        continue;
                    }
                    ++read;
                    if (iabs(cu[j][q]) == t[j]) {
                        lose |= 1u << j;
                        done |= 1u << j;
                    }
                    if (cu[j][q] > 0) seen[j] |= 1u << pos[j][q];
                }
                if (pull_only ? q0 + C >= len[j] : pm[j] == 0) done |= 1u << j;
            }
            if ((done & ((1u << K) - 1)) == (1u << K) - 1) break;
        }
        if (!pull_only) {
    #pragma unroll
            for (int j = 0; j < K; ++j)
                if (seen[j]) atomicAnd(&d.pend[v[j]], ~seen[j]);
        }
        // losers: one shared-memory atomic per wavefront for their slots, one for their degrees
        lose &= act;
        const uint32_t win = act & ~lose;
        int nl = 0;
        int64_t ldeg = 0;
        uint64_t lm[K];
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            lm[j] = __ballot(lose >> j & 1u);
            nl += __popcll(lm[j]);
            ldeg += lose >> j & 1u ? len[j] : 0;
        }
        if (nl) {
            const int64_t dsum = wave_sum(ldeg);
            int slot = 0;
            if (lane == 0) {
                slot = atomicAdd(&s_cnt[kL], nl);
                atomicAdd(&s_deg[kL], (unsigned long long)dsum);
            }
            slot = __shfl(slot, 0);
            if (slot + nl > seg_cap) {  // cannot happen (see above); reported instead of written
                if (lane == 0) d.ct->seg_overflow = 1;
                lose = 0;
            }
    #pragma unroll
            for (int j = 0; j < K; ++j) {
                if (lose >> j & 1u) {
                    if (d.racy) d.c[v[j]] = 0;
                    if (!discard) list[seg_base + slot + __popcll(lm[j] & lanes_below())] = v[j];
                }
                slot += __popcll(lm[j]);
            }
        }
        // winners commit
    #pragma unroll
        for (int j = 0; j < K; ++j) {
            if (!(win >> j & 1u)) continue;
            d.c[v[j]] = t[j];
            un.u[kUPushEntries] += pull_only ? 0 : len[j];
        }
        un.u[kUCommits] += __popc(win);
        un.u[kUConflictNodes] += __popc(act);
        un.u[kUConflictEntries] += read;
        // push modes: bit t - 1 into every neighbour's color mask (t <= d + 1 <= 33), read first,
        // the atomic only where the bit is missing
        if (!pull_only && win) {
            for (int32_t q0 = 0;; q0 += C) {
                int32_t w[K][C];
    #pragma unroll
                for (int j = 0; j < K; ++j)
    #pragma unroll
                    for (int q = 0; q < C; ++q)
                        w[j][q] = (win >> j & 1u) && q0 + q < len[j] ? d.colidx[b[j] + q0 + q] + gb[j] : -1;
                uint64_t mw[K][C];
    #pragma unroll
                for (int j = 0; j < K; ++j)
    #pragma unroll
                    for (int q = 0; q < C; ++q) mw[j][q] = w[j][q] >= 0 ? d.mask[w[j][q]] : ~0ull;
                bool more = false;
    #pragma unroll
                for (int j = 0; j < K; ++j) {
                    const uint64_t bit = 1ull << ((t[j] - 1) & 63);
    #pragma unroll
                    for (int q = 0; q < C; ++q)
                        if (!(mw[j][q] & bit)) atomicOr((unsigned long long *)&d.mask[w[j][q]], (unsigned long long)bit);
                    more |= (win >> j & 1u) && q0 + C < len[j];
                }
                if (!more) break;
            }
        }
        if (d.grounds) {
            // per item j: lanes committing nodes of the same graph as the first committing lane
            // share one atomic
    #pragma unroll
            for (int j = 0; j < K; ++j) {
                const bool wj = win >> j & 1u;
                const int32_t g = wj ? d.gidx[v[j]] : -1;
                const uint64_t cm = __ballot(wj);
                if (!cm) continue;
                const int leader = __ffsll((unsigned long long)cm) - 1;
                const int32_t g0 = __shfl(g, leader);
                const uint64_t same = __ballot(wj && g == g0);
                if (lane == leader) {
                    atomicMax(&d.grounds[g0], r);
                    if (d.gleft) atomicSub(&d.gleft[g0], (int32_t)__popcll(same));
                }
                if (wj && g != g0) {
                    atomicMax(&d.grounds[g], r);
                    if (d.gleft) atomicSub(&d.gleft[g], 1);
                }
            }
        }
    }
}

template <class D>
__device__ __forceinline__ void assign_step(const D &d, const RoundIn &in, Units &un, int G) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)G * blockDim.x;
    const int64_t gw = gt / kWave, nw = nt / kWave;
    const int lane = lane_id();
    // class L: a lane per node, several nodes in flight per lane
    if (in.topo) light_assign<true>(d, in.cv[kL], in.split, un, G);
    else light_assign<false>(d, in.cv[kL], in.split, un, G);
    // classes W and M.  Large rounds (at least four W/M nodes per wavefront): a thread per node
    // for the first zero bit of the color mask; nodes whose mask is full (64 colors taken) are
    // queued in shared memory and each gets a wavefront for its byte map from color 65 on (the
    // loop bounds depend on the workgroup only).  Small rounds: a wavefront per node.
    __shared__ int32_t s_full[kRoundBlock];
    __shared__ int s_nfull;
    const int32_t nW = in.cv[kW].total, nWM = nW + in.cv[kM].total;
    if ((int64_t)nWM >= 4 * nw) {
        if (threadIdx.x == 0) s_nfull = 0;
        __syncthreads();
        for (int64_t i0 = (int64_t)blockIdx.x * blockDim.x; i0 < nWM; i0 += nt) {
            const int64_t i = i0 + threadIdx.x;
            int32_t v = -1;
            bool full = false;
            if (i < nWM) {
                v = i < nW ? in.cv[kW].at((int32_t)i) : in.cv[kM].at((int32_t)(i - nW));
                const int32_t cv = d.c[v];
                if (!skip_item(d, in, v, cv)) {
                    const uint64_t free = ~d.mask[v];
                    un.u[kUMapBytes] += 8;
                    if (free) {
                        d.c[v] = -__ffsll((unsigned long long)free);
                        un.u[kUAssignNodes] += 1;
                    } else {
                        full = true;
                    }
                }
            }
            const int pos = block_append(full, &s_nfull);
            if (full) s_full[pos] = v;
            __syncthreads();
            for (int k = threadIdx.x / kWave; k < s_nfull; k += kRoundWaves) map_assign_wave(d, s_full[k], un);
            __syncthreads();
            if (threadIdx.x == 0) s_nfull = 0;
            __syncthreads();
        }
    } else {
        for (int64_t i = gw; i < nWM; i += nw) {
            const int32_t v = i < nW ? in.cv[kW].at((int32_t)i) : in.cv[kM].at((int32_t)(i - nW));
            const int32_t cv = d.c[v];
            if (skip_item(d, in, v, cv)) continue;
            const uint64_t free = ~d.mask[v];
            un.u[kUMapBytes] += lane == 0 ? 8 : 0;
            if (free) {
                if (lane == 0) {
                    d.c[v] = -__ffsll((unsigned long long)free);
                    un.u[kUAssignNodes] += 1;
                }
                continue;
            }
            map_assign_wave(d, v, un);
        }
    }
    un.fold();
}

// ============================================================== step 2: conflicts, commit, push
//
// v loses iff a smaller neighbour u holds the same tentative color (the lower
// id keeps its color).  Winners commit; W and L winners write their color into
// the byte maps of their neighbours at once, M winners are recorded for the
// push step; losers go to the workgroup's segment of the out list.

// Record color t with the neighbours in row entries [b, e) (neighbour ids
// offset by `base`, their byte maps by `fsh`), `width` threads with ranks
// `rank` (a wavefront or a team of them), four independent loads in flight per
// thread.  Colors up to 64 set a bit of the neighbour's mask: a read first,
// the atomic only if the bit is not set yet (a hub's word takes the same color
// from many winners).  Larger colors go to byte maps, skipping committed
// neighbours (which never read their maps again), class L neighbours when they
// read colors themselves, and maps too short for t.
template <class D>
__device__ __forceinline__ void push_row(const D &d, int64_t b, int64_t e, int32_t t, int32_t base, int64_t fsh,
                                         int rank, int width) {
    if (t <= kMaskColors) {
        const uint64_t bit = 1ull << (t - 1);
        for (int64_t k0 = b; k0 < e; k0 += 4 * width) {
            int32_t w[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int64_t k = k0 + j * width + rank;
                w[j] = k < e ? d.colidx[k] + base : -1;
            }
            uint64_t mw[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) mw[j] = w[j] >= 0 ? d.mask[w[j]] : bit;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (!(mw[j] & bit)) atomicOr((unsigned long long *)&d.mask[w[j]], (unsigned long long)bit);
        }
        return;
    }
    for (int64_t k0 = b; k0 < e; k0 += 4 * width) {
        int32_t w[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t k = k0 + j * width + rank;
            w[j] = k < e ? d.colidx[k] + base : -1;
        }
        bool skip[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // both loads are issued before either is tested
            const int32_t cw = w[j] >= 0 ? d.c[w[j]] : 1;
            const int8_t kw = w[j] >= 0 && d.light_pull == kPullLight ? d.cls[w[j]] : (int8_t)kW;
            skip[j] = cw > 0 || kw == kL;
        }
        MapRef fm[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) fm[j] = skip[j] ? MapRef{0, 0} : map_of(d, w[j], fsh);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((uint32_t)t <= fm[j].size) d.F[fm[j].pos + t - 1] = 1;
    }
}

template <class D>
__device__ __forceinline__ void push_row_wave(const D &d, int64_t b, int64_t e, int32_t t, int32_t base,
                                              int64_t fsh) {
    push_row(d, b, e, t, base, fsh, lane_id(), kWave);
}

// Ring scan of W/M node v by one wavefront: looks for a smaller neighbour with
// tentative color t, drops committed neighbours, keeps the others (moved to the
// ring's end) and advances the ring start past every entry it read.  The first
// pass reads one chunk of 64 entries, later passes `wide` (1..4) chunks, with as
// many independent loads in flight per lane; stops after the pass in which a
// conflict shows up.  Wide passes pay off in small, latency-bound rounds; in
// large rounds the extra entries a loser reads cost more bandwidth than they
// save in latency.  Kept entries are written past the ring's end, which never
// reaches an entry not yet read: at most `read` entries are kept and the ring
// never holds more than d entries.
// S = 64 or 16 lanes (a wavefront, or a quarter of one) scan node v's ring; the
// lanes of the group agree on every loop condition, and ballots are masked to
// the group.  Quarter-wave groups read four chunks of 16 entries per pass.
template <class D>
__device__ __forceinline__ bool ring_scan_group(const D &d, int32_t v, int32_t t, int wide, int S, Units &un) {
    constexpr int kPass = 4;
    const int lane = lane_id(), gl = lane % S;
    const uint64_t gm = S == kWave ? ~0ull : (((1ull << S) - 1) << (lane - gl));
    const int64_t base = d.rowptr[v];
    const int32_t cap = (int32_t)(d.rowptr[v + 1] - base);
    int32_t start = d.lstart[v], len = d.llen[v];
    int32_t read = 0, kept = 0;
    bool lose = false;
    int chunks = S == kWave ? 1 : kPass;  // a wavefront's first pass reads one chunk (a loser often stops there)
    while (read < len && !lose) {
        int32_t u[kPass], cu[kPass];
#pragma unroll
        for (int j = 0; j < kPass; ++j) {
            const int32_t k = read + j * S + gl;
            u[j] = -1;
            if (j < chunks && k < len) {
                int32_t p = start + k;
                if (p >= cap) p -= cap;
                u[j] = d.lower[base + p];
            }
        }
#pragma unroll
        for (int j = 0; j < kPass; ++j) cu[j] = u[j] >= 0 ? d.c[u[j]] : 0;
        bool hit = false;
#pragma unroll
        for (int j = 0; j < kPass; ++j) {
            hit |= u[j] >= 0 && iabs(cu[j]) == t;
            const bool keep = u[j] >= 0 && cu[j] <= 0;  // not committed (0: uncolored in place)
            const uint64_t km = __ballot(keep) & gm;
            if (keep) {
                int32_t p = start + len + kept + __popcll(km & lanes_below());
                while (p >= cap) p -= cap;
                d.lower[base + p] = u[j];
            }
            kept += __popcll(km);
        }
        lose = (__ballot(hit) & gm) != 0;
        read += min(chunks * S, len - read);
        if (S == kWave) chunks = wide;
    }
    un.u[kUConflictEntries] += gl == 0 ? read : 0;
    un.u[kUListWrites] += gl == 0 ? kept : 0;
    if (gl == 0 && len > 0) {
        int32_t s2 = start + read;
        while (s2 >= cap) s2 -= cap;
        d.lstart[v] = s2;
        d.llen[v] = len - read + kept;
    }
    return lose;
}


// Conflict test of the W/M nodes by teams of T wavefronts (T = 2, 4, 8 or 16)
// for rounds with few of them, so a long ring is read up to T times faster
// than by one wavefront: a pass reads 4 * T * 64 entries.  The teams of a
// workgroup run their passes together (the pass loop ends when none of them
// has entries left), so its workgroup barriers are uniform.  Kept entries
// are placed through a shared counter per team, so their order in the ring
// varies; the set, and with it every outcome, does not.
template <class D>
__device__ __forceinline__ void conflict_wide_teams(const D &d, const RoundIn &in, const OutSegs &os, int32_t r, Units &un, int G, int T,
                                    bool discard, const int64_t (&seg_base)[kNumClasses], int *s_cnt,
                                    unsigned long long *s_deg) {
    constexpr int kPass = 4;
    __shared__ int32_t s_kept[kRoundWaves], s_hit[kRoundWaves];
    const int span = T * kWave, tpb = kRoundWaves / T;
    const int tm = threadIdx.x / span, tl = threadIdx.x % span, lane = lane_id();
    const int64_t nteams = (int64_t)G * tpb;
    const int32_t nW = in.cv[kW].total, nWM = nW + in.cv[kM].total;
    // the slot loop depends on the workgroup only
    for (int64_t i0 = (int64_t)blockIdx.x * tpb; i0 < nWM; i0 += nteams) {
        const int64_t i = i0 + tm;
        const bool hub = i >= nW;
        int32_t v = 0, t = 0, start = 0, len = 0, cap = 0;
        int64_t b = 0, e = 0;
        bool act = i < nWM;
        if (act) {
            v = hub ? in.cv[kM].at((int32_t)(i - nW)) : in.cv[kW].at((int32_t)i);
            const int32_t cv = d.c[v];
            act = !skip_item(d, in, v, cv);
            t = -cv;
            b = d.rowptr[v];
            e = d.rowptr[v + 1];
            cap = (int32_t)(e - b);
            start = d.lstart[v];
            len = d.llen[v];
        }
        if (tl == 0) {
            s_kept[tm] = 0;
            s_hit[tm] = 0;
        }
        __syncthreads();
        int32_t read = 0;  // the same in every thread of a team
        bool scanning = act && len > 0;
        while (__syncthreads_or(scanning)) {
            int32_t u[kPass], cu[kPass];
#pragma unroll
            for (int j = 0; j < kPass; ++j) {
                const int32_t k = read + j * span + tl;
                u[j] = -1;
                if (scanning && k < len) {
                    int32_t p = start + k;
                    if (p >= cap) p -= cap;
                    u[j] = d.lower[b + p];
                }
            }
#pragma unroll
            for (int j = 0; j < kPass; ++j) cu[j] = u[j] >= 0 ? d.c[u[j]] : 0;
            bool hit = false;
#pragma unroll
            for (int j = 0; j < kPass; ++j) hit |= u[j] >= 0 && iabs(cu[j]) == t;
            __syncthreads();  // every read of the pass is done before kept entries reuse ring slots
#pragma unroll
            for (int j = 0; j < kPass; ++j) {
                const bool keep = u[j] >= 0 && cu[j] <= 0;
                const uint64_t km = __ballot(keep);
                int wb = 0;
                if (lane == 0 && km) wb = atomicAdd(&s_kept[tm], (int)__popcll(km));
                wb = __shfl(wb, 0);
                if (keep) {
                    int32_t p = start + len + wb + (int32_t)__popcll(km & lanes_below());
                    while (p >= cap) p -= cap;
                    d.lower[b + p] = u[j];
                }
            }
            if (hit) s_hit[tm] = 1;
            __syncthreads();
            if (scanning) {
                read += min(kPass * span, len - read);
                scanning = read < len && s_hit[tm] == 0;
            }
        }
        const bool lose = act && s_hit[tm] != 0;
        if (act && tl == 0) {
            const int32_t kept = s_kept[tm];
            un.u[kUConflictNodes] += 1;
            un.u[kUConflictEntries] += read;
            un.u[kUListWrites] += kept;
            if (len > 0) {
                int32_t s2 = start + read;
                while (s2 >= cap) s2 -= cap;
                d.lstart[v] = s2;
                d.llen[v] = len - read + kept;
            }
            const int q = hub ? kM : kW;
            if (lose) {
                if (d.racy) d.c[v] = 0;
                const int p = atomicAdd(&s_cnt[q], 1);
                atomicAdd(&s_deg[q], (unsigned long long)(e - b));
                if (!discard) os.list[seg_base[q] + p] = v;
            } else {
                d.c[v] = t;
                un.u[kUCommits] += 1;
                if (d.grounds) atomicMax(&d.grounds[d.gidx[v]], r);
                if (d.gleft) atomicSub(&d.gleft[d.gidx[v]], 1);
                if (hub) d.hub_won[atomicAdd(&d.ct->hub_winners, 1)] = HubRec{b, e, d.fshift(v), t, d.base(v)};
            }
        }
        if (act && !lose && !hub) {
            push_row(d, b, e, t, d.base(v), d.fshift(v), tl, span);
            if (tl == 0) un.u[kUPushEntries] += e - b;
        }
        __syncthreads();  // the team counters are reset for the next slot
    }
}

// Conflict test, commit and push of W/M node v (item of class W, or M if hub) by a group of S
// lanes (this lane is gl of them).
template <class D>
__device__ __forceinline__ void wide_conflict_item(const D &d, const RoundIn &in, const OutSegs &os, int32_t r, Units &un,
                                                   int32_t v, int32_t cv, bool hub, int S, int gl, bool discard,
                                                   const int64_t (&seg_base)[kNumClasses], int *s_cnt,
                                                   unsigned long long *s_deg) {
    const int32_t t = -cv;
    const bool lose = ring_scan_group(d, v, t, in.total <= kWideScanMax ? 4 : 1, S, un);
    const int64_t b = d.rowptr[v], e = d.rowptr[v + 1];
    const int q = hub ? kM : kW;
    if (gl == 0) un.u[kUConflictNodes] += 1;
    if (lose) {
        if (gl == 0) {
            if (d.racy) d.c[v] = 0;
            const int p = atomicAdd(&s_cnt[q], 1);
            atomicAdd(&s_deg[q], (unsigned long long)(e - b));
            if (!discard) os.list[seg_base[q] + p] = v;
        }
    } else {
        if (gl == 0) {
            d.c[v] = t;
            un.u[kUCommits] += 1;
            if (d.grounds) atomicMax(&d.grounds[d.gidx[v]], r);
            if (d.gleft) atomicSub(&d.gleft[d.gidx[v]], 1);
        }
        if (hub) {
            if (gl == 0) d.hub_won[atomicAdd(&d.ct->hub_winners, 1)] = HubRec{b, e, d.fshift(v), t, d.base(v)};
        } else {
            push_row(d, b, e, t, d.base(v), d.fshift(v), gl, S);
            un.u[kUPushEntries] += gl == 0 ? e - b : 0;
        }
    }
}

// part: 0 the round's only pass; 1 and 2 the two passes of a round of both kinds (per-graph
// schedules), whose losers share the workgroup's out segments: the first clears the counts, the
// second writes them.
template <class D>
__device__ __forceinline__ void conflict_step(const D &d, const RoundIn &in, const OutSegs &os, int32_t r, Units &un, int G,
                                              int part = 0) {
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (int64_t)G * blockDim.x;
    const int64_t gw = gt / kWave, nw = nt / kWave;
    const int lane = lane_id();
    __shared__ int s_cnt[kNumClasses];
    __shared__ unsigned long long s_deg[kNumClasses];
    if (part != 2 && threadIdx.x < kNumClasses) {
        s_cnt[threadIdx.x] = 0;
        s_deg[threadIdx.x] = 0;
    }
    __syncthreads();
    const bool discard = d.discard && in.topo;  // discard mode: a sweep keeps only the losers' count
    const int64_t seg_base[kNumClasses] = {os.cls_off[kL] + (int64_t)blockIdx.x * os.cap[kL],
                                           os.cls_off[kW] + (int64_t)blockIdx.x * os.cap[kW],
                                           os.cls_off[kM] + (int64_t)blockIdx.x * os.cap[kM]};

    // classes W and M: a wavefront per node.  W winners write their color into
    // their neighbours' byte maps at once; M winners are recorded for the push step.
    const int32_t nW = in.cv[kW].total, nWM = nW + in.cv[kM].total;
    int T = 1;  // wavefronts per W/M node: more when there are few of them
    while (T < kRoundWaves && (int64_t)nWM * T * 2 <= nw) T *= 2;
    if (T > 1) conflict_wide_teams(d, in, os, r, un, G, T, discard, seg_base, s_cnt, s_deg);
    // Without teams: a wavefront per node, or, when W nodes are many (at least four per
    // wavefront), a quarter wavefront per W node so that four latency chains overlap.
    const bool quarter = T == 1 && (int64_t)nW >= 4 * nw;
    for (int ph = 0; ph < 2 && T == 1; ++ph) {
        const int64_t cnt = ph == 0 && quarter ? nW : nWM - nW;  // nodes of this phase's class(es)
        const int S = ph == 0 && !quarter ? kWave : cnt >= 8 * nw ? 8 : cnt >= 4 * nw ? 16 : kWave;
        const int64_t lo = ph == 0 ? 0 : (quarter ? nW : nWM), hi = ph == 0 && quarter ? nW : nWM;
        const int per = kWave / S, gl = lane % S;
        if constexpr (kSplitDev<D>) {
            if (in.split && in.topo) {
                // the sweep of a round of both kinds: each lane judges one of the wavefront's next 64
                // items (iteration lane / per, slot lane % per), and the groups take only the kept ones
                const int64_t step = nw * per;
                for (int64_t w0 = lo + gw * per; w0 < hi; w0 += (int64_t)(kWave / per) * step) {
                    const int64_t ij = w0 + (int64_t)(lane / per) * step + lane % per;
                    int32_t vj = 0, cj = 0;
                    bool need = false;
                    if (ij < hi) {
                        vj = ij >= nW ? in.cv[kM].at((int32_t)(ij - nW)) : in.cv[kW].at((int32_t)ij);
                        cj = d.c[vj];
                        need = !skip_item(d, in, vj, cj);
                    }
                    const int hj = ij >= nW ? 1 : 0;
                    uint64_t nm = __ballot(need);
                    while (nm) {  // the same for the whole wavefront
                        uint64_t mm = nm;
                        for (int q = lane / S; q > 0 && mm; --q) mm &= mm - 1;
                        const int src = mm ? __ffsll((unsigned long long)mm) - 1 : 0;
                        const int32_t v = __shfl(vj, src), cv = __shfl(cj, src);
                        const bool hub = __shfl(hj, src) != 0;
                        for (int q = 0; q < per && nm; ++q) nm &= nm - 1;
                        if (mm) wide_conflict_item(d, in, os, r, un, v, cv, hub, S, gl, discard, seg_base, s_cnt, s_deg);
                    }
                }
                continue;
            }
        }
        // the loop is the same for the whole wavefront; group lane / S takes item i0 + lane / S
        for (int64_t i0 = lo + gw * per; i0 < hi; i0 += nw * per) {
            const int64_t i = i0 + lane / S;
            if (i >= hi) continue;
            const bool hub = i >= nW;
            const int32_t v = hub ? in.cv[kM].at((int32_t)(i - nW)) : in.cv[kW].at((int32_t)i);
            const int32_t cv = d.c[v];
            if (skip_item(d, in, v, cv)) continue;
            wide_conflict_item(d, in, os, r, un, v, cv, hub, S, gl, discard, seg_base, s_cnt, s_deg);
        }
    }
    // class L: a lane per node, several nodes in flight per lane
    if (in.topo) light_conflict<true>(d, in.cv[kL], in.split, seg_base[kL], discard, r, un, G, os.list, os.cap[kL], s_cnt, s_deg);
    else light_conflict<false>(d, in.cv[kL], in.split, seg_base[kL], discard, r, un, G, os.list, os.cap[kL], s_cnt, s_deg);
    __syncthreads();
    if (part != 1 && threadIdx.x < kNumClasses) {
        os.cnt[threadIdx.x * gridDim.x + blockIdx.x] = s_cnt[threadIdx.x];
        os.deg[threadIdx.x * gridDim.x + blockIdx.x] = (int64_t)s_deg[threadIdx.x];
    }
    un.fold();
}

// Push step: the rows of this round's committed hubs, spread over every
// wavefront of the grid in chunks of 256 entries.  Each workgroup stages up to
// kRoundBlock hubs at a time (row bounds, color, chunk prefix sums) in shared
// memory; wavefront w then takes chunks w, w + nw, ... of the staged batch.
template <class D>
__device__ __forceinline__ void hub_push_step(const D &d, int32_t nwon, Units &un, int G) {
    constexpr int kChunk = 4 * kWave;
    __shared__ int64_t s_b[kRoundBlock], s_e[kRoundBlock], s_fsh[kRoundBlock];
    __shared__ int32_t s_t[kRoundBlock], s_base[kRoundBlock], s_pre[kRoundBlock + 1];
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)G * blockDim.x / kWave;
    for (int32_t h0 = 0; h0 < nwon; h0 += blockDim.x) {
        const int32_t h = h0 + threadIdx.x;
        int32_t chunks = 0;
        if (h < nwon) {
            const HubRec rec = d.hub_won[h];
            s_b[threadIdx.x] = rec.b;
            s_e[threadIdx.x] = rec.e;
            s_t[threadIdx.x] = rec.t;
            s_base[threadIdx.x] = rec.base;
            s_fsh[threadIdx.x] = rec.fsh;
            chunks = (int32_t)((rec.e - rec.b + kChunk - 1) / kChunk);
        }
        int total;
        const int ex = block_scan(chunks, &total);
        s_pre[threadIdx.x] = ex;
        if (threadIdx.x == 0) s_pre[blockDim.x] = total;
        __syncthreads();
        const int nh = min((int32_t)blockDim.x, nwon - h0);
        for (int64_t g = gw; g < total; g += nw) {
            int lo = 0, hi = nh;  // hub lo with s_pre[lo] <= g < s_pre[lo + 1]
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_pre[mid] <= g) lo = mid;
                else hi = mid;
            }
            const int64_t k0 = s_b[lo] + (g - s_pre[lo]) * kChunk;
            push_row_wave(d, k0, min<int64_t>(k0 + kChunk, s_e[lo]), s_t[lo], s_base[lo], s_fsh[lo]);
            if (lane_id() == 0) un.u[kUPushEntries] += min<int64_t>(k0 + kChunk, s_e[lo]) - k0;
        }
        __syncthreads();
    }
    un.fold();
}

// ============================================================== round kernels

// Round bookkeeping by workgroup 0 (all its threads): trace, work units, and
// the stop test (a round that starts with an empty worklist is not run).
template <class D>
__device__ __forceinline__ void round_record(const D &d, int r, const RoundIn &in, bool reset_hubs, int writers) {
    __shared__ unsigned long long s_deg[kNumClasses];
    if (in.total == 0) {
        if (threadIdx.x == 0) {
            d.ct->finished = 1;
            d.ct->rounds = r - 1;
        }
        return;
    }
    if (threadIdx.x < kNumClasses) s_deg[threadIdx.x] = 0;
    __syncthreads();
    if (r > 1) {
        for (int k = 0; k < kNumClasses; ++k) {
            const int64_t x = threadIdx.x < (unsigned)writers ? d.seg_deg[r & 1][k * gridDim.x + threadIdx.x] : 0;
            const int64_t ws = wave_sum(x);
            if (lane_id() == 0 && ws) atomicAdd(&s_deg[k], (unsigned long long)ws);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t dsum = 0;
        for (int k = 0; k < kNumClasses; ++k) {
            const int64_t ds = r == 1 ? d.ct->class_deg[k] : (int64_t)s_deg[k];
            dsum += ds;
            d.ct->unit_nodes[k] += in.wl[k];
            d.ct->unit_edges[k] += ds;
        }
        if (r - 1 < d.trace_cap) {
            d.trace[r - 1] = in.total;
            d.trace_deg[r - 1] = dsum;
        }
        if (reset_hubs) {
            d.ct->hub_winners = 0;
            d.ct->prev_discarded = d.discard && in.topo;
        }
    }
}

template <class D>
__device__ __forceinline__ OutSegs out_segs(const D &d, int r) {
    OutSegs os;
    const int dst = (r + 1) & 1;  // round r writes the list round r+1 reads
    os.list = d.seg_list[dst];
    os.cnt = d.seg_cnt[dst];
    os.deg = d.seg_deg[dst];
    for (int k = 0; k < kNumClasses; ++k) {
        os.cls_off[k] = d.ct->seg_off[k];
        os.cap[k] = d.ct->seg_cap[k];
    }
    return os;
}

template <class D>
__device__ __forceinline__ void tick(const D &d, int64_t i) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && i < d.tick_cap) d.ticks[i] = wall_clock64();
}

// Discard mode, first data-driven round after sweeps: rebuild the worklist
// (list `par`) from the static lists.  Workgroup b takes items
// [b*span_k, (b+1)*span_k) of class k and appends its uncolored nodes, in
// order, to its own segment.
template <class D>
__device__ __forceinline__ void rebuild_step(const D &d, int par, int G) {
    __shared__ int s_cnt;
    __shared__ unsigned long long s_deg;
    const int b = blockIdx.x, nb = G, stride = gridDim.x;
    for (int k = 0; k < kNumClasses; ++k) {
        if (threadIdx.x == 0) {
            s_cnt = 0;
            s_deg = 0;
        }
        __syncthreads();
        const int32_t total = d.ct->class_n[k];
        const bool ident = d.ct->static_ident;
        const int32_t *list = d.static_list + d.ct->static_off[k];
        const int64_t span = ((int64_t)total + nb - 1) / nb, lo = (int64_t)b * span, hi = min<int64_t>(lo + span, total);
        int32_t *seg = d.seg_list[par] + d.ct->seg_off[k] + (int64_t)b * d.ct->seg_cap[k];  // segment b of class k
        for (int64_t c0 = lo; c0 < hi; c0 += blockDim.x) {
            const int64_t i = c0 + threadIdx.x;
            const int32_t v = i >= hi ? 0 : ident ? (int32_t)(d.ct->static_off[k] + i) : list[i];
            const bool act = i < hi && d.c[v] <= 0;
            const int64_t ds = wave_sum(act ? d.rowptr[v + 1] - d.rowptr[v] : 0);
            if (lane_id() == 0 && ds) atomicAdd(&s_deg, (unsigned long long)ds);
            const int p = block_append(act, &s_cnt);
            if (act) seg[p] = v;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            d.seg_cnt[par][k * stride + b] = s_cnt;
            d.seg_deg[par][k * stride + b] = (int64_t)s_deg;
        }
        __syncthreads();
    }
}

// Workgroups for a data-driven round with `total` active nodes, given the
// `G` of the previous round: all of them, until the worklist has at most
// kTailNodesPerGroup nodes per tail workgroup; then tail_groups of them (at
// most one node per thread, so no workgroup's out segment can overflow).
// Fewer participants make each grid barrier cheaper (every workgroup's
// agent-scope acquire is part of its cost); the worklist only shrinks, so G
// never grows again.
constexpr int kTailNodesPerGroup = 32;

template <class D>
__device__ __forceinline__ int round_groups(const D &d, const RoundIn &in, int G) {
    if (in.topo || d.tail_groups <= 0 || G <= d.tail_groups) return G;
    return (int64_t)in.total <= (int64_t)d.tail_groups * kTailNodesPerGroup ? d.tail_groups : G;
}

// Per-graph schedules, round r > 1: the view of the first pass (the worklist, or the static list
// when no graph runs data-driven), and whether a sweeping second pass follows.
template <class D>
__device__ __forceinline__ RoundIn graph_round(const D &d, int r, int32_t (*pre)[kMaxRoundBlocks + 1], Split sp,
                                               bool *two) {
    *two = sp.topo > 0 && sp.data > 0;
    RoundIn in = round_view(d, r, pre, sp.topo > 0 && sp.data == 0 ? 1 : 0);
    in.split = *two;
    return in;
}

// The second pass of a round of both kinds: the static list, nodes of topology-driven graphs.
template <class D>
__device__ __forceinline__ RoundIn sweep_view(const D &d, int r, int32_t (*pre)[kMaxRoundBlocks + 1]) {
    RoundIn in = round_view(d, r, pre, 1);
    in.split = true;
    return in;
}

// Rounds first .. last (or until the worklist is empty) in one cooperative
// launch: assign | barrier | conflict | barrier [| hub push | barrier].  Every
// workgroup reads the same counts after each barrier, so all take the same
// branches and leave the loop together; in the tail of the run, workgroups
// G and up leave it early (round_groups) and the barrier counts the rest.
// Round 1 reads the static list; a later first round reads the segmented
// list of its parity, written by every workgroup.
template <class D>
__global__ __launch_bounds__(kRoundBlock) void k_rounds(D d, int32_t first, int32_t last) {
    __shared__ int32_t pre[kNumClasses][kMaxRoundBlocks + 1];
    GridBarrier gb;
    const bool up = gb.setup(d.bar, d.bar_limit);
    Units un;
    if (!up || input_bad(d.ct)) last = first - 1;  // a wait gave up, or unusable input: leave at once
    int32_t r = first;
    int G = gridDim.x;        // workgroups in the round loop
    int writers = gridDim.x;  // workgroups that wrote the list this round reads
    bool discarded = false;   // the previous round kept no worklist
    for (; r <= last; ++r) {
        if (r > 1) load_segments(d, r & 1, pre, writers);
        RoundIn in = round_view(d, r, pre);
        bool two = false;  // per-graph schedules: a round of both kinds (a second, sweeping pass)
        if constexpr (kSplitDev<D>) {
            if (d.gthr) {
                // every workgroup reads gleft before the assign barrier, so before any commit of round r
                Split sp{0, 0};
                if (r == 1) {
                    if (blockIdx.x == 0) sp = graph_split(d, true);
                } else {
                    sp = graph_split(d, false);
                    if (sp.topo == 0) {
                        // gleft only shrinks, so every graph stays data-driven from here on: the rounds
                        // left go to the plain batch kernel, which carries none of this code
                        if (blockIdx.x == 0 && threadIdx.x == 0) d.ct->resume_round = r;
                        break;
                    }
                }
                if (r > 1) in = graph_round(d, r, pre, sp, &two);
                if (blockIdx.x == 0 && threadIdx.x == 0 && r - 1 < d.topo_cap) d.trace_topo[r - 1] = sp.topo;
            }
        }
        if (discarded && !in.topo && in.total > 0) {
            rebuild_step(d, r & 1, G);
            if (!gb.sync()) break;
            writers = G;
            load_segments(d, r & 1, pre, writers);
            in = round_view(d, r, pre);
        }
        discarded = d.discard && in.topo;
        if (blockIdx.x == 0) round_record(d, r, in, false, writers);
        if (in.total == 0) break;
        // a round of both kinds keeps every workgroup: its sweep spreads the whole static list
        const int g2 = two ? G : round_groups(d, in, G);
        if (g2 < G) {
            if ((int)blockIdx.x >= g2) break;
            gb.shrink(g2);
            G = g2;
        }
        tick(d, 3 * (int64_t)(r - 1));
        if (r > 1) {  // round 1's tentative colors (all 1) were set at init
            assign_step(d, in, un, G);
            if (two) assign_step(d, sweep_view(d, r, pre), un, G);
            if (!gb.sync()) break;
        }
        tick(d, 3 * (int64_t)(r - 1) + 1);
        conflict_step(d, in, out_segs(d, r), r, un, G, two ? 1 : 0);
        if (two) conflict_step(d, sweep_view(d, r, pre), out_segs(d, r), r, un, G, 2);
        writers = G;
        if (!gb.sync()) break;
        tick(d, 3 * (int64_t)(r - 1) + 2);
        // every workgroup reads the count here (one load, shared); it is cleared only after the next barrier
        __shared__ int32_t s_nwon;
        if (threadIdx.x == 0) s_nwon = (int32_t)ld_agent((unsigned *)&d.ct->hub_winners);
        __syncthreads();
        const int32_t nwon = s_nwon;
        if (nwon > 0) {
            hub_push_step(d, nwon, un, G);
            if (!gb.sync()) break;
            if (blockIdx.x == 0 && threadIdx.x == 0) d.ct->hub_winners = 0;
        }
    }
    tick(d, 3 * (int64_t)(r - 1));
    un.flush(d);
}

// The same steps as separate launches (the launch boundary is the barrier),
// for hosts that cannot launch cooperatively and for per-step timing.
// Stepped launches, discard mode: the rebuild of round r when round r - 1 kept no worklist.
template <class D>
__global__ __launch_bounds__(kRoundBlock) void k_rebuild_round(D d, int32_t r) {
    if (d.ct->finished || r == 1 || !d.ct->prev_discarded || input_bad(d.ct)) return;
    __shared__ int32_t pre[kNumClasses][kMaxRoundBlocks + 1];
    load_segments(d, r & 1, pre, gridDim.x);
    const RoundIn in = round_view(d, r, pre);
    if (in.topo || in.total == 0) return;
    rebuild_step(d, r & 1, gridDim.x);
}

template <class D>
__global__ __launch_bounds__(kRoundBlock) void k_assign_round(D d, int32_t r) {
    if (d.ct->finished || input_bad(d.ct)) return;
    __shared__ int32_t pre[kNumClasses][kMaxRoundBlocks + 1];
    if (r > 1) load_segments(d, r & 1, pre, gridDim.x);
    RoundIn in = round_view(d, r, pre);
    bool two = false;
    if constexpr (kSplitDev<D>) {
        if (d.gthr) {  // per-graph schedules: decided here, from gleft before any commit of round r
            Split sp{0, 0};
            if (r > 1 || blockIdx.x == 0) sp = graph_split(d, r == 1);
            if (r > 1) in = graph_round(d, r, pre, sp, &two);
            if (blockIdx.x == 0) {  // for this round's conflict launch
                if (threadIdx.x == 0) {
                    d.ct->split_topo = sp.topo;
                    d.ct->split_data = sp.data;
                    if (r - 1 < d.topo_cap) d.trace_topo[r - 1] = sp.topo;
                }
                for (int w = threadIdx.x; w < (d.ngraphs + 63) / 64 * 2; w += blockDim.x) d.gsplit[w] = graph_bits()[w];
            }
        }
    }
    if (blockIdx.x == 0) round_record(d, r, in, true, gridDim.x);
    if (in.total == 0 || r == 1) return;  // round 1's tentative colors were set at init
    Units un;
    assign_step(d, in, un, gridDim.x);
    if (two) assign_step(d, sweep_view(d, r, pre), un, gridDim.x);
    un.flush(d);
}

template <class D>
__global__ __launch_bounds__(kRoundBlock) void k_conflict_round(D d, int32_t r) {
    if (d.ct->finished || input_bad(d.ct)) return;
    __shared__ int32_t pre[kNumClasses][kMaxRoundBlocks + 1];
    if (r > 1) load_segments(d, r & 1, pre, gridDim.x);
    RoundIn in = round_view(d, r, pre);
    bool two = false;
    if constexpr (kSplitDev<D>) {
        if (d.gthr && r > 1) {  // the decision of this round's assign launch
            const Split sp{d.ct->split_topo, d.ct->split_data};
            in = graph_round(d, r, pre, sp, &two);
            if (two) {
                for (int w = threadIdx.x; w < (d.ngraphs + 63) / 64 * 2; w += blockDim.x) graph_bits()[w] = d.gsplit[w];
                __syncthreads();
            }
        }
    }
    if (in.total == 0) return;
    Units un;
    conflict_step(d, in, out_segs(d, r), r, un, gridDim.x, two ? 1 : 0);
    if (two) conflict_step(d, sweep_view(d, r, pre), out_segs(d, r), r, un, gridDim.x, 2);
    un.flush(d);
}

// Round 1 of a graph whose nodes are all of class L and pull their neighbours' colors (so the static
// list is the identity), as a launch of its own before the cooperative round kernel, which then
// starts at round 2.  Every node holds tentative color 1, so node v loses iff it has a smaller
// neighbour: with sorted rows the row's first entry decides, otherwise the whole row is read; no
// state is read.  Winners commit color 1; losers go to this workgroup's class-L segment, as the
// round kernel's round 1 leaves them.  Blocks of 64 * K nodes go round the workgroups of the round
// kernel's grid, so no workgroup takes more than n / G + 64 * K * (1 + 1/G) nodes: its segment holds
// them.  Eight nodes per lane keep many row reads in flight (this step has no other work).
template <class D>
__global__ __launch_bounds__(kRoundBlock) void k_round1_light(D d) {
    constexpr int K = 8;
    static_assert(2 * kWave * K <= kRoundBlock, "a workgroup's share fits its out segment");
    if (input_bad(d.ct)) return;
    __shared__ int32_t pre[kNumClasses][kMaxRoundBlocks + 1];  // not read: round 1 reads the static list
    __shared__ int s_cnt;
    __shared__ unsigned long long s_deg;
    const RoundIn in = round_view(d, 1, pre);
    if (blockIdx.x == 0) round_record(d, 1, in, true, gridDim.x);
    const int64_t n = in.cv[kL].total;
    if (in.total == 0) return;
    tick(d, 0);
    tick(d, 1);
    Units un;
    if (threadIdx.x == 0) {
        s_cnt = 0;
        s_deg = 0;
    }
    __syncthreads();
    const OutSegs os = out_segs(d, 1);
    const int64_t seg = os.cls_off[kL] + (int64_t)blockIdx.x * os.cap[kL];
    const int lane = lane_id();
    const int64_t gw = (int64_t)(threadIdx.x / kWave) * gridDim.x + blockIdx.x;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t b0 = gw * (kWave * K); b0 < n; b0 += nw * (kWave * K)) {
        int64_t a[K], e[K];
        uint32_t act = 0, lose = 0;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int64_t v = b0 + j * kWave + lane;
            act |= (v < n ? 1u : 0u) << j;
            a[j] = v < n ? (int64_t)d.rowptr[v] : 0;
            e[j] = v < n ? (int64_t)d.rowptr[v + 1] : 0;
        }
        int32_t read = 0;
        if (d.sorted) {  // the first entry is the row's smallest
            int64_t u[K];
#pragma unroll
            for (int j = 0; j < K; ++j) u[j] = a[j] < e[j] ? (int64_t)d.colidx[a[j]] + d.base((int32_t)(b0 + j * kWave + lane)) : INT64_MAX;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                lose |= (u[j] < b0 + j * kWave + lane ? 1u : 0u) << j;
                read += a[j] < e[j];
            }
        } else {
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const int64_t v = b0 + j * kWave + lane;
                const int64_t base = v < n ? d.base((int32_t)v) : 0;
                for (int64_t k0 = a[j]; k0 < e[j]; k0 += 4) {
                    int64_t u[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) u[q] = k0 + q < e[j] ? (int64_t)d.colidx[k0 + q] + base : INT64_MAX;
                    bool hit = false;
#pragma unroll
                    for (int q = 0; q < 4; ++q) hit |= u[q] < v;
                    read += (int32_t)min<int64_t>(4, e[j] - k0);
                    if (hit) {
                        lose |= 1u << j;
                        break;
                    }
                }
            }
        }
        lose &= act;
        // losers: one shared-memory atomic per wavefront for their slots, one for their degrees
        int nl = 0;
        int64_t ldeg = 0;
        uint64_t lm[K];
#pragma unroll
        for (int j = 0; j < K; ++j) {
            lm[j] = __ballot(lose >> j & 1u);
            nl += __popcll(lm[j]);
            ldeg += lose >> j & 1u ? e[j] - a[j] : 0;
        }
        if (nl) {
            const int64_t dsum = wave_sum(ldeg);
            int slot = 0;
            if (lane == 0) {
                slot = atomicAdd(&s_cnt, nl);
                atomicAdd(&s_deg, (unsigned long long)dsum);
            }
            slot = __shfl(slot, 0);
            if (slot + nl > os.cap[kL]) {  // cannot happen (see above); reported instead of written
                if (lane == 0) d.ct->seg_overflow = 1;
            } else {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    if (lose >> j & 1u) os.list[seg + slot + __popcll(lm[j] & lanes_below())] = (int32_t)(b0 + j * kWave + lane);
                    slot += __popcll(lm[j]);
                }
            }
        }
        // winners commit color 1
        const uint32_t win = act & ~lose;
#pragma unroll
        for (int j = 0; j < K; ++j)
            if (win >> j & 1u) d.c[b0 + j * kWave + lane] = 1;
        un.u[kUCommits] += __popc(win);
        un.u[kUConflictNodes] += __popc(act);
        un.u[kUConflictEntries] += read;
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses) {
        os.cnt[threadIdx.x * gridDim.x + blockIdx.x] = threadIdx.x == kL ? s_cnt : 0;
        os.deg[threadIdx.x * gridDim.x + blockIdx.x] = threadIdx.x == kL ? (int64_t)s_deg : 0;
    }
    un.flush(d);
}

template <class D>
__global__ __launch_bounds__(kRoundBlock) void k_push_round(D d) {
    if (d.ct->finished || input_bad(d.ct)) return;
    const int32_t nwon = d.ct->hub_winners;
    if (nwon == 0) return;
    Units un;
    hub_push_step(d, nwon, un, gridDim.x);
    un.flush(d);
}

}  // namespace ipgc
