// IPGC graph coloring for MI355X (gfx950): HIP kernels and the C-ABI driver.
//
// Method: Section II-C of Rai, M P, Pai, "A Hybrid Graph Coloring Algorithm for
// GPUs" (arXiv 1912.01478): rounds of (1) first-fit tentative coloring of every
// uncolored node and (2) uncoloring one endpoint of each edge whose endpoints
// picked the same color.  Schedule: Section IV, a worklist of uncolored nodes is
// kept in every round, and each round runs topology-driven (sweep over all
// nodes, active nodes found by their state) or data-driven (over the worklist),
// chosen by comparing the worklist size with the threshold H.
//
// State layout (one int32 per node, kept in the caller's output buffer):
//   c[v] > 0   v holds committed color c[v];
//   c[v] <= 0  v is uncolored; after the assign step of a round it holds -t,
//              where t >= 1 is its tentative color for that round.
// The sign encoding gives the synchronous semantics without a second array:
//   * assign reads neighbours' c[u] and counts only c[u] > 0, so a neighbour
//     writing its own -t concurrently is invisible either way;
//   * conflict compares |c[u]| with v's tentative t.  A neighbour committed in
//     an earlier round holds a color that was forbidden to v, so it never
//     equals t; a neighbour active in this round holds -t_u or, once it wins,
//     +t_u, and |c[u]| = t_u in both cases.  No membership test is needed.
//
// Nodes are split by degree into three buckets, each with its own kernel shape:
//   light  (deg <= light_max, at most 63): one thread per node, forbidden
//          colors in a 64-bit register (a node of degree d can only see d
//          colors, so its color is at most d + 1 <= 64);
//   wave   (deg <= wave_max, at most 2047): one wavefront per node, lanes read
//          the row with unit stride, forbidden colors in a per-wave LDS bitmap
//          of 2048 bits;
//   block  (larger): one workgroup per node, LDS bitmap of 65536 colors per
//          pass (further passes only if a node sees 65536 distinct colors).
// Worklist pushes are aggregated per wavefront with a ballot, one atomic add
// per wave instead of one per node.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "ipgc.h"

namespace {

constexpr int kWave = 64;
constexpr int kLightBlock = 256;
constexpr int kWaveBlock = 256;               // 4 wavefronts, one node each at a time
constexpr int kWavesPerBlock = kWaveBlock / kWave;
constexpr int kWaveBitmapWords = 64;          // 2048 colors: covers every wave-bucket node
constexpr int kMaxWaveDegree = kWaveBitmapWords * 32 - 1;
constexpr int kBlockThreads = 256;
constexpr int kBlockBitmapWords = 2048;       // 65536 colors per pass
constexpr int kDefaultLightMax = 32;
constexpr int kDefaultWaveMax = 1024;
constexpr int kMaxGrid = 16384;

enum { kLight = 0, kWaveB = 1, kBlockB = 2, kNumBuckets = 3 };
enum { kStatic = 0, kListA = 1, kListB = 2, kNumLists = 3 };

// Device-resident counters, one set per workspace.
struct Counters {
    int64_t deg[kNumLists][4];   // degree sum of the entries per bucket in each list
    int64_t unit_nodes[4];       // active nodes processed per bucket, summed over rounds
    int64_t unit_edges[4];       // their degree sums, summed over rounds
    int32_t size[kNumLists][4];  // entries per bucket in each list
    int32_t off[4];              // bucket region offsets, identical in every list buffer
    int32_t fill[4];             // cursors while filling the static list
    int32_t finished;            // 1 once a round left the worklist empty
    int32_t rounds;              // rounds run when finished
    int32_t bad_rows;            // rows with decreasing pointers or pointers outside [0, m]
    int32_t bad_ids;             // column ids outside [0, n)
    int32_t unsorted_rows;       // rows not strictly ascending
    int32_t pad[3];
};

struct GraphArgs {
    const int32_t *rowptr;
    const int32_t *colidx;
    int32_t *c;
    int32_t n;
    int32_t light_max;
    int32_t sorted;
};

struct RoundArgs {
    const int32_t *in_list;      // worklist read by data-driven rounds (bucket regions)
    int32_t *out_list;           // worklist written with the round's losers
    const int32_t *static_list;  // every node by bucket (the topology sweep of wave and block buckets)
    int32_t in;                  // list index of in_list (for its counters)
    int32_t out;                 // list index of out_list
    int32_t round;               // 1-based
    int64_t threshold;           // topology round iff |WL| > threshold
    int32_t *trace;              // |WL_r| per round
    int64_t *trace_deg;          // sum of degrees over WL_r per round
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t lanes_below() {
    int l = lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ int32_t wl_total(const Counters *ct, int list) {
    return ct->size[list][0] + ct->size[list][1] + ct->size[list][2];
}

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Append `v` (degree `d`) to bucket `b` of `out_list` for every lane with
// `push` set; one atomic per wavefront for the slots and one for the degree
// sum.  Must be called by all lanes of the wave.
__device__ __forceinline__ void wave_push(bool push, int32_t v, int32_t d, int b, Counters *ct, int out, int32_t *out_list) {
    uint64_t mask = __ballot(push);
    if (mask == 0) return;
    int leader = __ffsll((unsigned long long)mask) - 1;
    int64_t dsum = wave_sum(push ? (int64_t)d : 0);
    int base = 0;
    if (lane_id() == leader) {
        base = atomicAdd(&ct->size[out][b], __popcll(mask));
        atomicAdd((unsigned long long *)&ct->deg[out][b], (unsigned long long)dsum);
    }
    base = __shfl(base, leader);
    if (push) out_list[ct->off[b] + base + __popcll(mask & lanes_below())] = v;
}

// ------------------------------------------------------------------ init and validation

// c[v] = 0 for every node (Section II-C: all nodes start uncolored and in the
// worklist), row pointer checks, and bucket sizes of the static list.
__global__ __launch_bounds__(kLightBlock) void k_init(GraphArgs g, int32_t m, int32_t wave_max, Counters *ct) {
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < g.n; base += stride) {
        int v = base + threadIdx.x;
        int b = -1;
        bool bad = false;
        if (v < g.n) {
            g.c[v] = 0;
            int32_t lo = g.rowptr[v], hi = g.rowptr[v + 1];
            bad = lo < 0 || hi < lo || hi > m;
            int32_t d = bad ? 0 : hi - lo;
            b = d <= g.light_max ? kLight : (d <= wave_max ? kWaveB : kBlockB);
        }
        const int64_t dv = (v < g.n && !bad) ? (int64_t)(g.rowptr[v + 1] - g.rowptr[v]) : 0;
        for (int k = 0; k < kNumBuckets; ++k) {
            uint64_t mask = __ballot(b == k);
            int64_t dsum = wave_sum(b == k ? dv : 0);
            if (mask && lane_id() == __ffsll((unsigned long long)mask) - 1) {
                atomicAdd(&ct->size[kStatic][k], __popcll(mask));
                atomicAdd((unsigned long long *)&ct->deg[kStatic][k], (unsigned long long)dsum);
            }
        }
        uint64_t badmask = __ballot(bad);
        if (badmask && lane_id() == 0) atomicAdd(&ct->bad_rows, __popcll(badmask));
    }
}

__global__ void k_offsets(Counters *ct) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ct->off[0] = 0;
        ct->off[1] = ct->size[kStatic][0];
        ct->off[2] = ct->off[1] + ct->size[kStatic][1];
        ct->off[3] = ct->off[2] + ct->size[kStatic][2];
        for (int b = 0; b < 4; ++b) ct->fill[b] = 0;
    }
}

__global__ __launch_bounds__(kLightBlock) void k_fill_static(GraphArgs g, int32_t wave_max, Counters *ct, int32_t *static_list) {
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < g.n; base += stride) {
        int v = base + threadIdx.x;
        int b = -1;
        if (v < g.n) {
            int32_t d = g.rowptr[v + 1] - g.rowptr[v];
            b = d <= g.light_max ? kLight : (d <= wave_max ? kWaveB : kBlockB);
        }
        for (int k = 0; k < kNumBuckets; ++k) {
            uint64_t mask = __ballot(b == k);
            if (mask == 0) continue;
            int leader = __ffsll((unsigned long long)mask) - 1;
            int pos = 0;
            if (lane_id() == leader) pos = atomicAdd(&ct->fill[k], __popcll(mask));
            pos = __shfl(pos, leader);
            if (b == k) static_list[ct->off[k] + pos + __popcll(mask & lanes_below())] = v;
        }
    }
}

// Column checks: every id in [0, n), and whether rows are strictly ascending.
// Light rows: a thread per row.
__global__ __launch_bounds__(kLightBlock) void k_check_light(GraphArgs g, Counters *ct, const int32_t *static_list) {
    const int count = ct->size[kStatic][kLight];
    const int32_t *list = static_list + ct->off[kLight];
    int bad = 0, unsorted = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        int v = list[i];
        int32_t prev = -1;
        for (int32_t k = g.rowptr[v]; k < g.rowptr[v + 1]; ++k) {
            int32_t u = g.colidx[k];
            bad += (u < 0 || u >= g.n);
            unsorted |= (u <= prev);
            prev = u;
        }
    }
    uint64_t bm = __ballot(bad != 0), um = __ballot(unsorted != 0);
    if (lane_id() == 0 && bm) atomicAdd(&ct->bad_ids, __popcll(bm));
    if (lane_id() == 0 && um) atomicAdd(&ct->unsorted_rows, __popcll(um));
}

// Wave and block rows: a wavefront per row, lanes with unit stride.
__global__ __launch_bounds__(kWaveBlock) void k_check_wide(GraphArgs g, Counters *ct, const int32_t *static_list) {
    const int count = ct->size[kStatic][kWaveB] + ct->size[kStatic][kBlockB];
    const int32_t *list = static_list + ct->off[kWaveB];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    int bad = 0, unsorted = 0;
    for (int i = blockIdx.x * kWavesPerBlock + wave; i < count; i += gridDim.x * kWavesPerBlock) {
        int v = list[i];
        int32_t b = g.rowptr[v], e = g.rowptr[v + 1];
        for (int32_t k = b + lane; k < e; k += kWave) {
            int32_t u = g.colidx[k];
            bad += (u < 0 || u >= g.n);
            if (k + 1 < e) unsorted |= (g.colidx[k + 1] <= u);
        }
    }
    uint64_t bm = __ballot(bad != 0), um = __ballot(unsorted != 0);
    if (lane_id() == 0 && bm) atomicAdd(&ct->bad_ids, __popcll(bm));
    if (lane_id() == 0 && um) atomicAdd(&ct->unsorted_rows, __popcll(um));
}

// ------------------------------------------------------------------ step 1: tentative first-fit colors

// The smallest color >= 1 that no committed neighbour holds (footnote on mex in
// Section II-C; colors are 1-based because 0 marks an uncolored node).

__device__ __forceinline__ bool round_header(const Counters *ct, const RoundArgs &rd, bool &topo, int32_t &total) {
    if (ct->finished) return false;
    total = wl_total(ct, rd.in);
    topo = (int64_t)total > rd.threshold;
    return total > 0;
}

__global__ __launch_bounds__(kLightBlock) void k_assign_light(GraphArgs g, RoundArgs rd, Counters *ct) {
    bool topo;
    int32_t total;
    if (!round_header(ct, rd, topo, total)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rd.trace[rd.round - 1] = total;
        int64_t dsum = 0;
        for (int b = 0; b < kNumBuckets; ++b) {
            dsum += ct->deg[rd.in][b];
            ct->unit_nodes[b] += ct->size[rd.in][b];
            ct->unit_edges[b] += ct->deg[rd.in][b];
            // The out list of this round was the in list of the previous round; nothing reads it any more.
            ct->size[rd.out][b] = 0;
            ct->deg[rd.out][b] = 0;
        }
        rd.trace_deg[rd.round - 1] = dsum;
    }
    const int count = topo ? g.n : ct->size[rd.in][kLight];
    const int32_t *list = rd.in_list + ct->off[kLight];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        int v;
        if (topo) {
            v = i;
            if (g.c[v] > 0) continue;                                  // committed: not active
            if (g.rowptr[v + 1] - g.rowptr[v] > g.light_max) continue;  // handled by a wider kernel
        } else {
            v = list[i];
        }
        uint64_t used = 0;
        for (int32_t k = g.rowptr[v]; k < g.rowptr[v + 1]; ++k) {
            int32_t cu = g.c[g.colidx[k]];
            if (cu > 0 && cu <= 64) used |= 1ull << (cu - 1);
        }
        g.c[v] = -(__ffsll((unsigned long long)~used));  // degree <= 63 leaves a zero bit
    }
}

__global__ __launch_bounds__(kWaveBlock) void k_assign_wave(GraphArgs g, RoundArgs rd, Counters *ct) {
    bool topo;
    int32_t total;
    if (!round_header(ct, rd, topo, total)) return;
    __shared__ uint32_t bitmap[kWavesPerBlock][kWaveBitmapWords];
    const int wave = threadIdx.x / kWave, lane = lane_id();
    uint32_t *bm = bitmap[wave];
    const int count = topo ? ct->size[kStatic][kWaveB] : ct->size[rd.in][kWaveB];
    const int32_t *list = (topo ? rd.static_list : rd.in_list) + ct->off[kWaveB];
    for (int i = blockIdx.x * kWavesPerBlock + wave; i < count; i += gridDim.x * kWavesPerBlock) {
        int v = list[i];
        if (topo && g.c[v] > 0) continue;
        const int32_t b = g.rowptr[v], e = g.rowptr[v + 1], d = e - b;
        const int words = d / 32 + 1;  // colors 1..d+1 map to bits 0..d
        bm[lane] = 0;
        wave_sync();
        for (int32_t k = b + lane; k < e; k += kWave) {
            int32_t cu = g.c[g.colidx[k]];
            if (cu > 0 && cu <= d + 1) atomicOr(&bm[(cu - 1) >> 5], 1u << ((cu - 1) & 31));
        }
        wave_sync();
        uint32_t word = lane < words ? bm[lane] : 0u;
        uint64_t free_words = __ballot(word != 0xffffffffu);
        int first = __ffsll((unsigned long long)free_words) - 1;  // exists: the color is at most d + 1
        uint32_t fw = __shfl(word, first < 0 ? 0 : first);
        if (lane == 0) g.c[v] = first < 0 ? -(d + 1) : -(first * 32 + __ffs(~fw));
        wave_sync();
    }
}

__global__ __launch_bounds__(kBlockThreads) void k_assign_block(GraphArgs g, RoundArgs rd, Counters *ct) {
    bool topo;
    int32_t total;
    if (!round_header(ct, rd, topo, total)) return;
    __shared__ uint32_t bm[kBlockBitmapWords];
    __shared__ int s_first;
    const int count = topo ? ct->size[kStatic][kBlockB] : ct->size[rd.in][kBlockB];
    const int32_t *list = (topo ? rd.static_list : rd.in_list) + ct->off[kBlockB];
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        int v = list[i];
        const int32_t cv = g.c[v];
        __syncthreads();  // every thread has read c[v] before thread 0 may overwrite it
        if (topo && cv > 0) continue;
        const int32_t b = g.rowptr[v], e = g.rowptr[v + 1], d = e - b;
        // Pass p covers colors [base + 1, base + 65536]; the answer is at most d + 1.
        for (int64_t base = 0; base <= d; base += 32 * kBlockBitmapWords) {
            const int64_t span = std::min<int64_t>((int64_t)d + 1 - base, 32 * kBlockBitmapWords);
            const int words = (int)((span + 31) / 32);
            for (int w = threadIdx.x; w < words; w += blockDim.x) bm[w] = 0;
            if (threadIdx.x == 0) s_first = INT32_MAX;
            __syncthreads();
            for (int32_t k = b + threadIdx.x; k < e; k += blockDim.x) {
                int64_t cu = (int64_t)g.c[g.colidx[k]] - base;
                if (cu > 0 && cu <= span) atomicOr(&bm[(cu - 1) >> 5], 1u << ((cu - 1) & 31));
            }
            __syncthreads();
            for (int w = threadIdx.x; w < words; w += blockDim.x) {
                uint32_t word = bm[w];
                if (w == words - 1 && (span & 31)) word |= ~0u << (span & 31);  // bits past the span
                if (word != 0xffffffffu) atomicMin(&s_first, w * 32 + __ffs(~word) - 1);
            }
            __syncthreads();
            const int first = s_first;
            __syncthreads();
            if (first != INT32_MAX) {
                if (threadIdx.x == 0) g.c[v] = -(int32_t)(base + first + 1);
                break;
            }
        }
    }
}

// ------------------------------------------------------------------ step 2: conflicts, commit, worklist push

// v loses iff some neighbour u < v holds the same tentative color (reading R4:
// the lower id keeps its color).  Winners commit, losers go to the out list.

__global__ __launch_bounds__(kLightBlock) void k_conflict_light(GraphArgs g, RoundArgs rd, Counters *ct) {
    bool topo;
    int32_t total;
    if (!round_header(ct, rd, topo, total)) return;
    const int count = topo ? g.n : ct->size[rd.in][kLight];
    const int32_t *list = rd.in_list + ct->off[kLight];
    const int stride = gridDim.x * blockDim.x;
    for (int base = blockIdx.x * blockDim.x; base < count; base += stride) {  // wave-uniform loop
        const int i = base + threadIdx.x;
        bool lose = false;
        int v = 0;
        int32_t d = 0;
        if (i < count) {
            bool active = true;
            if (topo) {
                v = i;
                active = g.c[v] < 0 && g.rowptr[v + 1] - g.rowptr[v] <= g.light_max;
            } else {
                v = list[i];
            }
            if (active) {
                const int32_t t = -g.c[v];
                d = g.rowptr[v + 1] - g.rowptr[v];
                for (int32_t k = g.rowptr[v]; k < g.rowptr[v + 1]; ++k) {
                    int32_t u = g.colidx[k];
                    if (u >= v) {
                        if (g.sorted) break;
                        continue;
                    }
                    int32_t cu = g.c[u];
                    if (cu == t || cu == -t) { lose = true; break; }
                }
                if (!lose) g.c[v] = t;
            }
        }
        wave_push(lose, v, d, kLight, ct, rd.out, rd.out_list);
    }
}

__global__ __launch_bounds__(kWaveBlock) void k_conflict_wave(GraphArgs g, RoundArgs rd, Counters *ct) {
    bool topo;
    int32_t total;
    if (!round_header(ct, rd, topo, total)) return;
    const int wave = threadIdx.x / kWave, lane = lane_id();
    const int count = topo ? ct->size[kStatic][kWaveB] : ct->size[rd.in][kWaveB];
    const int32_t *list = (topo ? rd.static_list : rd.in_list) + ct->off[kWaveB];
    for (int i = blockIdx.x * kWavesPerBlock + wave; i < count; i += gridDim.x * kWavesPerBlock) {
        const int v = list[i];
        const int32_t cv = g.c[v];
        if (topo && cv > 0) continue;
        const int32_t t = -cv;
        const int32_t b = g.rowptr[v], e = g.rowptr[v + 1];
        bool lose = false;
        for (int32_t k0 = b; k0 < e; k0 += kWave) {
            const int32_t k = k0 + lane;
            bool hit = false, past = false;
            if (k < e) {
                int32_t u = g.colidx[k];
                if (u < v) {
                    int32_t cu = g.c[u];
                    hit = (cu == t || cu == -t);
                } else {
                    past = true;
                }
            }
            if (__ballot(hit)) { lose = true; break; }
            if (g.sorted && __ballot(past)) break;
        }
        if (lane == 0) {
            if (lose) {
                int pos = atomicAdd(&ct->size[rd.out][kWaveB], 1);
                atomicAdd((unsigned long long *)&ct->deg[rd.out][kWaveB], (unsigned long long)(e - b));
                rd.out_list[ct->off[kWaveB] + pos] = v;
            } else {
                g.c[v] = t;
            }
        }
    }
}

__global__ __launch_bounds__(kBlockThreads) void k_conflict_block(GraphArgs g, RoundArgs rd, Counters *ct) {
    bool topo;
    int32_t total;
    if (!round_header(ct, rd, topo, total)) return;
    const int count = topo ? ct->size[kStatic][kBlockB] : ct->size[rd.in][kBlockB];
    const int32_t *list = (topo ? rd.static_list : rd.in_list) + ct->off[kBlockB];
    for (int i = blockIdx.x; i < count; i += gridDim.x) {
        const int v = list[i];
        const int32_t cv = g.c[v];
        __syncthreads();  // every thread has read c[v] before thread 0 may overwrite it
        if (topo && cv > 0) continue;
        const int32_t t = -cv;
        const int32_t b = g.rowptr[v], e = g.rowptr[v + 1];
        bool lose = false;
        for (int32_t k0 = b; k0 < e; k0 += blockDim.x) {
            const int32_t k = k0 + threadIdx.x;
            int hit = 0, past = 0;
            if (k < e) {
                int32_t u = g.colidx[k];
                if (u < v) {
                    int32_t cu = g.c[u];
                    hit = (cu == t || cu == -t);
                } else {
                    past = 1;
                }
            }
            if (__syncthreads_or(hit)) { lose = true; break; }
            if (g.sorted && __syncthreads_or(past)) break;
        }
        if (threadIdx.x == 0) {
            if (lose) {
                int pos = atomicAdd(&ct->size[rd.out][kBlockB], 1);
                atomicAdd((unsigned long long *)&ct->deg[rd.out][kBlockB], (unsigned long long)(e - b));
                rd.out_list[ct->off[kBlockB] + pos] = v;
            } else {
                g.c[v] = t;
            }
        }
        __syncthreads();
    }
}

// Round end: the loop stops once a round leaves the worklist empty (Section
// II-C); later enqueued rounds see `finished` and do nothing.
__global__ void k_round_end(RoundArgs rd, Counters *ct) {
    if (threadIdx.x != 0 || blockIdx.x != 0 || ct->finished) return;
    if (wl_total(ct, rd.out) == 0) {
        ct->finished = 1;
        ct->rounds = rd.round;
    }
}

// ------------------------------------------------------------------ host side

thread_local char g_err[512];

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(IPGC_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Profile kernel kinds (ipgc_kernel_name).
enum Kind {
    kKindInit = 0, kKindCheck, kKindAssignLight, kKindAssignWave, kKindAssignBlock,
    kKindConflictLight, kKindConflictWave, kKindConflictBlock, kKindRoundEnd, kNumKinds
};
const char *const kKindNames[kNumKinds] = {
    "init", "check", "assign_light", "assign_wave", "assign_block",
    "conflict_light", "conflict_wave", "conflict_block", "round_end"};

struct Workspace {
    int32_t *lists = nullptr;     // kNumLists * cap_n
    int32_t *trace = nullptr;     // cap_n
    int64_t *trace_deg = nullptr; // cap_n
    Counters *ct = nullptr;
    Counters *host_ct = nullptr;  // pinned
    int64_t cap_n = 0;
    std::vector<hipEvent_t> events;  // profile event pool

    void free_buffers() {
        if (lists) (void)hipFree(lists);
        if (trace) (void)hipFree(trace);
        if (trace_deg) (void)hipFree(trace_deg);
        lists = nullptr;
        trace = nullptr;
        trace_deg = nullptr;
        cap_n = 0;
    }

    void release() {
        free_buffers();
        if (ct) (void)hipFree(ct);
        if (host_ct) (void)hipHostFree(host_ct);
        ct = nullptr;
        host_ct = nullptr;
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        events.clear();
    }

    int reserve(int64_t n) {
        if (!ct) {
            HIP_TRY(hipMalloc(&ct, sizeof(Counters)));
            HIP_TRY(hipHostMalloc(&host_ct, sizeof(Counters), hipHostMallocDefault));
        }
        if (n <= cap_n) return IPGC_OK;
        free_buffers();
        int64_t want = std::max<int64_t>(n, 1024);
        if (hipMalloc(&lists, sizeof(int32_t) * kNumLists * want) != hipSuccess ||
            hipMalloc(&trace, sizeof(int32_t) * want) != hipSuccess ||
            hipMalloc(&trace_deg, sizeof(int64_t) * want) != hipSuccess) {
            (void)hipGetLastError();
            free_buffers();
            return fail(IPGC_ENOMEM, "workspace of %lld nodes does not fit in device memory", (long long)want);
        }
        cap_n = want;
        return IPGC_OK;
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

// Brackets launches of the selected kernel kinds with HIP events on the call's stream.
struct Profiler {
    Workspace &ws;
    hipStream_t s;
    uint32_t mask;
    std::vector<int> kinds;  // kind of each recorded (start, stop) pair
    size_t used = 0;

    int begin(int kind) {
        if (!(mask >> kind & 1u)) return IPGC_OK;
        hipEvent_t e;
        int rc = ws.event(used, &e);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(e, s));
        ++used;
        return IPGC_OK;
    }
    int end(int kind) {
        if (!(mask >> kind & 1u)) return IPGC_OK;
        hipEvent_t e;
        int rc = ws.event(used, &e);
        if (rc) return rc;
        HIP_TRY(hipEventRecord(e, s));
        ++used;
        kinds.push_back(kind);
        return IPGC_OK;
    }
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

#define TRY(expr)                  \
    do {                           \
        int rc_ = (expr);          \
        if (rc_) return rc_;       \
    } while (0)

std::mutex g_mutex;
std::vector<Workspace> g_ws;

int grid_for(int64_t items, int per_block) {
    int64_t g = (items + per_block - 1) / per_block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, kMaxGrid));
}

int read_counters(Workspace &ws, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(ws.host_ct, ws.ct, sizeof(Counters), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return IPGC_OK;
}

int color_impl(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m, int mode,
               const ipgc_options *opt, hipStream_t s, int32_t *out_colors, int32_t *out_rounds, ipgc_trace *trace) {
    if (!out_rounds) return fail(IPGC_EINVAL, "out_rounds is NULL");
    *out_rounds = -1;
    if (n < 0 || m < 0) return fail(IPGC_EINVAL, "negative size (n=%lld, m=%lld)", (long long)n, (long long)m);
    if (mode != IPGC_MODE_TOPOLOGY && mode != IPGC_MODE_DATA && mode != IPGC_MODE_HYBRID)
        return fail(IPGC_EINVAL, "unknown mode %d", mode);
    if (n >= INT32_MAX || m >= INT32_MAX) return fail(IPGC_ETOOBIG, "n=%lld or m=%lld exceeds int32 CSR", (long long)n, (long long)m);
    ipgc_options o{};
    if (opt) o = *opt;
    if (o.reserved != 0) return fail(IPGC_EINVAL, "options.reserved must be 0");
    int light_max = o.light_max_degree ? o.light_max_degree : kDefaultLightMax;
    int wave_max = o.wave_max_degree ? o.wave_max_degree : kDefaultWaveMax;
    if (light_max < 1 || light_max > 63) return fail(IPGC_EINVAL, "light_max_degree %d outside 1..63", light_max);
    if (wave_max <= light_max || wave_max > kMaxWaveDegree)
        return fail(IPGC_EINVAL, "wave_max_degree %d outside %d..%d", wave_max, light_max + 1, kMaxWaveDegree);
    if (o.validate < IPGC_VALIDATE_DEFAULT || o.validate > IPGC_VALIDATE_RANGES)
        return fail(IPGC_EINVAL, "unknown validate level %d", o.validate);
    const bool check_ids = o.validate != IPGC_VALIDATE_NONE;
    ipgc_profile *prof = o.profile;
    if (prof) {
        const uint32_t mask = prof->mask;
        std::memset(prof, 0, sizeof *prof);
        prof->mask = mask;
        prof->kinds = kNumKinds;
    }
    if (trace) trace->recorded = 0;
    if (n == 0) {
        *out_rounds = 0;
        return IPGC_OK;
    }
    if (!rowptr || !out_colors || (m > 0 && !colidx)) return fail(IPGC_EINVAL, "null device pointer");
    int64_t H;
    if (mode == IPGC_MODE_TOPOLOGY) H = -1;          // |WL| > -1 always holds
    else if (mode == IPGC_MODE_DATA) H = INT64_MAX;  // never
    else H = o.threshold > 0 ? o.threshold : (6 * n) / 10;

    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mutex);
    if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
    Workspace &ws = g_ws[dev];
    TRY(ws.reserve(n));
    Profiler pf{ws, s, prof ? prof->mask : 0u, {}, 0};

    // rowptr[0] == 0 and rowptr[n] == m.
    int32_t ends[2];
    HIP_TRY(hipMemcpyAsync(&ends[0], rowptr, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&ends[1], rowptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ends[0] != 0 || ends[1] != m)
        return fail(IPGC_EBADCSR, "rowptr[0]=%d rowptr[n]=%d, expected 0 and m=%lld", ends[0], ends[1], (long long)m);

    int32_t *lists[kNumLists];
    for (int l = 0; l < kNumLists; ++l) lists[l] = ws.lists + (int64_t)l * ws.cap_n;

    GraphArgs g{rowptr, colidx, out_colors, (int32_t)n, light_max, 0};
    HIP_TRY(hipMemsetAsync(ws.ct, 0, sizeof(Counters), s));
    TRY(pf.begin(kKindInit));
    k_init<<<grid_for(n, kLightBlock), kLightBlock, 0, s>>>(g, (int32_t)m, wave_max, ws.ct);
    k_offsets<<<1, 1, 0, s>>>(ws.ct);
    TRY(pf.end(kKindInit));
    HIP_TRY(hipGetLastError());
    TRY(read_counters(ws, s));
    if (ws.host_ct->bad_rows) return fail(IPGC_EBADCSR, "%d rows have invalid row pointers", ws.host_ct->bad_rows);
    int32_t bucket_n[kNumBuckets];
    for (int b = 0; b < kNumBuckets; ++b) bucket_n[b] = ws.host_ct->size[kStatic][b];
    TRY(pf.begin(kKindInit));
    k_fill_static<<<grid_for(n, kLightBlock), kLightBlock, 0, s>>>(g, wave_max, ws.ct, lists[kStatic]);
    TRY(pf.end(kKindInit));
    if (check_ids) {
        TRY(pf.begin(kKindCheck));
        k_check_light<<<grid_for(bucket_n[kLight], kLightBlock), kLightBlock, 0, s>>>(g, ws.ct, lists[kStatic]);
        if (bucket_n[kWaveB] + bucket_n[kBlockB] > 0)
            k_check_wide<<<grid_for(bucket_n[kWaveB] + bucket_n[kBlockB], kWavesPerBlock), kWaveBlock, 0, s>>>(g, ws.ct, lists[kStatic]);
        TRY(pf.end(kKindCheck));
        HIP_TRY(hipGetLastError());
        TRY(read_counters(ws, s));
        if (ws.host_ct->bad_ids) return fail(IPGC_EBADCSR, "%d rows hold column ids outside [0, n)", ws.host_ct->bad_ids);
        g.sorted = ws.host_ct->unsorted_rows == 0;
    }
    HIP_TRY(hipGetLastError());

    // Rounds.  Round 1 reads the static list (every node); then A and B alternate.
    int64_t known_total = n;  // worklist size at the start of the next round
    int32_t known_sizes[kNumBuckets] = {bucket_n[0], bucket_n[1], bucket_n[2]};
    int32_t r = 0;
    for (;;) {
        ++r;
        if (r > n) return fail(IPGC_ELIMIT, "round limit exceeded");  // the worklist shrinks every round
        const int in = r == 1 ? kStatic : (r % 2 == 0 ? kListA : kListB);
        const int out = r % 2 == 1 ? kListA : kListB;
        RoundArgs rd{lists[in], lists[out], lists[kStatic], in, out, r, H, ws.trace, ws.trace_deg};
        const bool topo = known_total > H;
        const int64_t nl = topo ? n : known_sizes[kLight];
        const int64_t nw = topo ? bucket_n[kWaveB] : known_sizes[kWaveB];
        const int64_t nb = topo ? bucket_n[kBlockB] : known_sizes[kBlockB];
        TRY(pf.begin(kKindAssignLight));
        k_assign_light<<<grid_for(nl, kLightBlock), kLightBlock, 0, s>>>(g, rd, ws.ct);
        TRY(pf.end(kKindAssignLight));
        if (nw) {
            TRY(pf.begin(kKindAssignWave));
            k_assign_wave<<<grid_for(nw, kWavesPerBlock), kWaveBlock, 0, s>>>(g, rd, ws.ct);
            TRY(pf.end(kKindAssignWave));
        }
        if (nb) {
            TRY(pf.begin(kKindAssignBlock));
            k_assign_block<<<grid_for(nb, 1), kBlockThreads, 0, s>>>(g, rd, ws.ct);
            TRY(pf.end(kKindAssignBlock));
        }
        if (nl) {
            TRY(pf.begin(kKindConflictLight));
            k_conflict_light<<<grid_for(nl, kLightBlock), kLightBlock, 0, s>>>(g, rd, ws.ct);
            TRY(pf.end(kKindConflictLight));
        }
        if (nw) {
            TRY(pf.begin(kKindConflictWave));
            k_conflict_wave<<<grid_for(nw, kWavesPerBlock), kWaveBlock, 0, s>>>(g, rd, ws.ct);
            TRY(pf.end(kKindConflictWave));
        }
        if (nb) {
            TRY(pf.begin(kKindConflictBlock));
            k_conflict_block<<<grid_for(nb, 1), kBlockThreads, 0, s>>>(g, rd, ws.ct);
            TRY(pf.end(kKindConflictBlock));
        }
        TRY(pf.begin(kKindRoundEnd));
        k_round_end<<<1, 1, 0, s>>>(rd, ws.ct);
        TRY(pf.end(kKindRoundEnd));
        HIP_TRY(hipGetLastError());
        TRY(read_counters(ws, s));
        if (ws.host_ct->finished) break;
        for (int b = 0; b < kNumBuckets; ++b) known_sizes[b] = ws.host_ct->size[out][b];
        known_total = (int64_t)known_sizes[0] + known_sizes[1] + known_sizes[2];
    }
    const int32_t rounds = ws.host_ct->rounds;
    if (trace) {
        const int64_t k = std::min<int64_t>(trace->capacity, rounds);
        if (k > 0 && trace->wl_size)
            HIP_TRY(hipMemcpyAsync(trace->wl_size, ws.trace, sizeof(int32_t) * k, hipMemcpyDeviceToHost, s));
        if (k > 0 && trace->wl_degree)
            HIP_TRY(hipMemcpyAsync(trace->wl_degree, ws.trace_deg, sizeof(int64_t) * k, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (k > 0 && trace->topology && trace->wl_size)
            for (int64_t i = 0; i < k; ++i) trace->topology[i] = (int8_t)((int64_t)trace->wl_size[i] > H);
        trace->recorded = k;
    }
    if (prof) {
        HIP_TRY(hipStreamSynchronize(s));
        TRY(pf.collect(prof));
        const Counters &hc = *ws.host_ct;
        prof->nodes[kKindInit] = n;
        prof->edges[kKindInit] = 0;
        prof->nodes[kKindCheck] = check_ids ? n : 0;
        prof->edges[kKindCheck] = check_ids ? m : 0;
        for (int b = 0; b < kNumBuckets; ++b) {
            prof->nodes[kKindAssignLight + b] = prof->nodes[kKindConflictLight + b] = hc.unit_nodes[b];
            prof->edges[kKindAssignLight + b] = prof->edges[kKindConflictLight + b] = hc.unit_edges[b];
        }
        prof->nodes[kKindRoundEnd] = rounds;
    }
    *out_rounds = rounds;
    g_err[0] = 0;
    return IPGC_OK;
}

}  // namespace

extern "C" {

int ipgc_color_graph(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                     int32_t *out_colors, int32_t *out_rounds) {
    return color_impl(csr_rowptr, csr_colidx, n, m, mode, nullptr, nullptr, out_colors, out_rounds, nullptr);
}

int ipgc_color_graph_ex(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                        const ipgc_options *options, void *stream, int32_t *out_colors, int32_t *out_rounds,
                        ipgc_trace *trace) {
    return color_impl(csr_rowptr, csr_colidx, n, m, mode, options, (hipStream_t)stream, out_colors, out_rounds, trace);
}

const char *ipgc_last_error(void) { return g_err; }

const char *ipgc_kernel_name(int kind) { return kind >= 0 && kind < kNumKinds ? kKindNames[kind] : ""; }

int ipgc_version(void) { return (1 << 16) | 0; }

void ipgc_release_workspaces(void) {
    std::lock_guard<std::mutex> lock(g_mutex);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (size_t d = 0; d < g_ws.size(); ++d) {
        if (hipSetDevice((int)d) == hipSuccess) g_ws[d].release();
    }
    (void)hipSetDevice(cur);
    g_ws.clear();
}

}  // extern "C"
