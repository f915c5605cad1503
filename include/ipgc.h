/*
 * ipgc.h -- C ABI of the MI355X (gfx950) graph-coloring library.
 *
 * The library colors an undirected graph with IPGC, Iterative Parallel Graph
 * Coloring, as described in Section II-C of Rai, M P, Pai, "A Hybrid Graph
 * Coloring Algorithm for GPUs" (arXiv 1912.01478).  Each round assigns every
 * uncolored node the smallest color its colored neighbours do not hold, then
 * uncolors one endpoint of every edge whose endpoints picked the same color.
 * It repeats until no node is uncolored.  Rounds run either topology-driven
 * (a sweep over all nodes) or data-driven (over the worklist of uncolored
 * nodes).  The hybrid schedule of Section IV keeps the worklist in both kinds
 * of round and picks the kind from the worklist size against a threshold H.
 *
 * Semantics are fixed so that the result is deterministic and identical for
 * every schedule (Section V: all versions run the same algorithm and give the
 * same colors):
 *   - colors are 1-based; 0 never appears in the output;
 *   - rounds are synchronous: assignments read the colors committed before the
 *     round, and conflict tests read all of the round's tentative colors;
 *   - on a conflict the endpoint with the lower node id keeps its color;
 *   - a round is topology-driven iff the worklist size |WL| > H.
 * The output satisfies 1 <= color[v] <= deg(v) + 1, and the colors used are
 * exactly 1..max(color).
 *
 * Graph format: symmetric CSR with int32 row pointers (n + 1 entries, rowptr[0]
 * = 0, rowptr[n] = m) and int32 column indices (m entries, each in [0, n)),
 * where m counts both directions of every edge.  Self-loops and duplicate
 * entries change nothing in the result.  If every row is sorted ascending, the
 * library detects that and lets conflict scans stop at the first neighbour id
 * that is not smaller than the node's own.
 *
 * Threads: calls are serialized per device inside the library, which keeps
 * one cached workspace per device.  All functions return IPGC_OK (0) or a
 * negative ipgc_status; ipgc_last_error() then describes the failure.
 */
#ifndef IPGC_H
#define IPGC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ipgc_status {
    IPGC_OK = 0,
    IPGC_EINVAL = -1,   /* null pointer with n > 0, n < 0, m < 0, bad mode or options */
    IPGC_ETOOBIG = -2,  /* n or m does not fit the int32 CSR */
    IPGC_EBADCSR = -3,  /* rowptr[0] != 0, rowptr[n] != m, decreasing rowptr, or id out of [0, n) */
    IPGC_ENOMEM = -4,   /* device workspace allocation failed */
    IPGC_EHIP = -5,     /* a HIP runtime call failed, or a grid-barrier wait exceeded its time limit */
    IPGC_ELIMIT = -6,   /* the round limit was reached (cannot happen for valid input: rounds <= n) */
    IPGC_ECANCELED = -7 /* a server job was cancelled before it finished (ipgc_server_cancel) */
} ipgc_status;

/* Round schedules (Section IV).  TOPOLOGY runs every round as a sweep over all
 * nodes, DATA runs every round over the worklist, HYBRID picks per round with
 * the threshold H.  All three push the nodes that lose a conflict onto the
 * worklist.  REBUILD is the discard-and-rebuild hybrid the paper contrasts
 * its own with (Section I): rounds are picked as for HYBRID, but sweeps keep
 * no worklist, and the first data-driven round after sweeps rebuilds it by
 * scanning every node.  All four give the same colors and round count. */
typedef enum ipgc_mode {
    IPGC_MODE_TOPOLOGY = 0,
    IPGC_MODE_DATA = 1,
    IPGC_MODE_HYBRID = 2,
    IPGC_MODE_REBUILD = 3
} ipgc_mode;

/* Validation levels.  A column id outside [0, n) would make the kernels read
 * outside the color array, so the default checks every id.
 *
 * The method colors an undirected simple graph, and the experiments of Section V
 * remove self-loops and multi-edges first.  The kernels learn a node's forbidden
 * colors from pushes along its neighbours' rows, so on a CSR that is not
 * symmetric they would not follow the definition (which reads the node's own
 * row).  IPGC_VALIDATE_FULL rejects such input: every entry (v, u) needs its
 * reverse (u, v), and no row may hold v itself or the same id twice.  It sorts a
 * copy of every row in the library's workspace (rows already sorted are copied)
 * and looks each reverse entry up by binary search: O(m log max_degree) work on
 * the device, off the coloring's own path. */
enum {
    IPGC_VALIDATE_DEFAULT = 0, /* same as IPGC_VALIDATE_RANGES */
    IPGC_VALIDATE_NONE = 1,    /* trust the caller: only rowptr[0] == 0 and rowptr[n] == m are checked */
    IPGC_VALIDATE_RANGES = 2,  /* also rowptr non-decreasing and every column id in [0, n) */
    IPGC_VALIDATE_FULL = 3     /* also a simple symmetric graph: no self-loop, no duplicate entry in a row,
                                  and (u, v) present for every entry (v, u); IPGC_EBADCSR otherwise */
};

/* Kernel kinds that ipgc_profile can time (see ipgc_kernel_name) and work
 * unit kinds it reports (see ipgc_unit_name). */
#define IPGC_PROFILE_KINDS 16

/* Optional device-time profile of one call.  Kernel kinds whose bit is set in
 * `mask` are bracketed by HIP events recorded on the call's stream; event
 * times and launch counts are summed per kind.  `units` are work counts the
 * kernels keep on the device (active nodes handled, neighbour entries read,
 * ...), from which an algorithmic byte count follows.  Host memory owned by
 * the caller; every out field is overwritten. */
typedef struct ipgc_profile {
    uint32_t mask;                            /* in: bit k times kernel kind k */
    int32_t kinds;                            /* out: number of kernel kinds defined */
    double ms[IPGC_PROFILE_KINDS];            /* out: summed event time per kind */
    int64_t launches[IPGC_PROFILE_KINDS];     /* out: timed launches per kind */
    int32_t unit_kinds;                       /* out: number of work unit kinds defined */
    int32_t reserved;
    int64_t units[IPGC_PROFILE_KINDS];        /* out: work units of the whole call */
    uint64_t *phase_ticks;                    /* in: host array or NULL.  out: device wall-clock ticks at
                                                 the start of each round's assign and conflict steps
                                                 (3 per round: assign, conflict, hub push) and at the end */
    int64_t phase_capacity;                   /* in: entries available in phase_ticks */
    int64_t phase_recorded;                   /* out: entries written */
    int64_t tick_khz;                         /* out: rate of the tick counter */
} ipgc_profile;

/* Tuning options.  A zeroed struct (or NULL) selects every default.  No option
 * changes the result, only the time. */
typedef struct ipgc_options {
    int64_t threshold;         /* H for HYBRID (topology round iff |WL| > H); 0 or less: floor(6n/10), the
                                  paper's 60% of the node count.  Ignored by TOPOLOGY and DATA. */
    int32_t light_max_degree;  /* nodes with degree <= this run a thread each; the others a wavefront
                                  each (1..32; 0: default 32) */
    int32_t hub_min_degree;    /* nodes with degree above this are hubs: when one commits, the whole
                                  grid writes its color into its neighbours' byte maps in a separate
                                  step of the round (> light_max_degree; 0: default 1024) */
    int32_t validate;          /* IPGC_VALIDATE_* */
    int32_t flags;             /* IPGC_FLAG_* */
    ipgc_profile *profile;     /* optional per-kernel timing and work counts (NULL: none) */
    int32_t workgroups;        /* workgroups of the round kernels (0: one per 4096 nodes, at most what
                                  the device keeps resident at once; larger values are clamped to that) */
    int32_t tail_workgroups;   /* once a data-driven round has at most 32 * tail_workgroups active nodes,
                                  only this many workgroups stay in the cooperative round loop (cheaper
                                  grid barriers for the long tail of small rounds; 0: default, negative:
                                  all workgroups stay) */
    int32_t barrier_timeout_ms; /* limit on every grid-barrier wait of a cooperative launch: a workgroup
                                  that waits longer gives up, every other one leaves at its next wait,
                                  and the call returns IPGC_EHIP (0: default 60000; -1: give up at the
                                  first wait that does not complete at once, to exercise that path) */
    int32_t reserved;          /* must be 0 */
} ipgc_options;

/* Option flags. */
enum {
    IPGC_FLAG_STEPPED = 1,     /* one launch per round step instead of one cooperative launch for all
                                  rounds (same result; used for per-step timing) */
    IPGC_FLAG_LIGHT_PULL = 2,  /* nodes of degree <= light_max_degree read their neighbours' colors in
                                  every assign instead of receiving them in a byte map (same result) */
    IPGC_FLAG_LIGHT_PUSH = 4,  /* every committed color is written into every neighbour's byte map.
                                  Neither flag: pull when no node is above light_max_degree, else push */
    IPGC_FLAG_RACY = 8,        /* in-place mode: a node that loses a conflict uncolors at once (a later
                                  test in the same step no longer sees it) and light nodes also avoid
                                  their neighbours' visible tentative colors.  Fewer rounds, but the
                                  colors and round count depend on timing: the result is a proper
                                  coloring with colors in [1, deg+1], not the synchronous one.
                                  Implies IPGC_FLAG_LIGHT_PULL unless IPGC_FLAG_LIGHT_PUSH is given. */
    IPGC_FLAG_PER_GRAPH = 16   /* ipgc_color_graphs_batched: every graph takes the schedule decision on its
                                  own (see there).  The other entry points ignore it: for one graph the
                                  decision is the same either way. */
};

/* Per-round record, filled on request.  Host memory owned by the caller. */
typedef struct ipgc_trace {
    int64_t capacity;    /* entries available in each array below */
    int32_t *wl_size;    /* |WL_r| at the start of round r (r = 0 .. rounds-1), may be NULL */
    int64_t *wl_degree;  /* sum of the degrees of the nodes in WL_r, may be NULL */
    int8_t *topology;    /* 1 if round r ran topology-driven, 0 if data-driven, may be NULL (per-graph
                            batches: 1 if at least one graph ran it topology-driven) */
    int64_t recorded;    /* out: min(rounds, capacity) */
    int32_t *topo_graphs; /* batches with IPGC_FLAG_PER_GRAPH: number of graphs that ran round r
                            topology-driven, may be NULL (other calls leave it untouched) */
} ipgc_trace;

/*
 * Color a graph (Section II-C, schedule of Section IV).
 *
 * csr_rowptr  DEVICE pointer, n + 1 int32 entries (caller-owned, read only).
 * csr_colidx  DEVICE pointer, m int32 entries (caller-owned, read only).
 * n, m        node count and CSR entry count; 0 <= n < 2^31 - 1, 0 <= m < 2^31.
 * mode        an ipgc_mode.
 * out_colors  DEVICE pointer, n int32 entries (caller-owned).  The library uses
 *             it as its color state during the run; on success it holds the
 *             final 1-based colors.  On error its contents are unspecified.
 * out_rounds  HOST pointer: number of rounds run (-1 on error).
 *
 * Blocks until the colors are in out_colors.  Runs on the device that is
 * current for the calling thread, on its null stream.  n = 0 succeeds with
 * zero rounds.  The library keeps no caller pointer after returning.
 */
int ipgc_color_graph(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                     int32_t *out_colors, int32_t *out_rounds);

/*
 * As ipgc_color_graph, with options (NULL: defaults), a HIP stream (a
 * hipStream_t passed as void*; NULL: the null stream) on which all work is
 * enqueued, and an optional per-round trace (NULL: none).  Still blocks until
 * the result is complete, because out_rounds is host memory.
 */
int ipgc_color_graph_ex(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                        const ipgc_options *options, void *stream, int32_t *out_colors, int32_t *out_rounds,
                        ipgc_trace *trace);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * coloring as ipgc_color_graph_ex, with every piece of workspace carved from
 * one static device array of IPGC_NOALLOC_SCRATCH_BYTES that the library's
 * code object holds on each GPU it runs on (until the process ends).  The call
 * makes no hipMalloc, hipFree, pinned-host or event allocation; the caller
 * passes the CSR and out_colors as for ipgc_color_graph_ex.
 *
 * The workspace of a graph takes about 46 bytes per node, 5 bytes per CSR
 * entry (9 with IPGC_VALIDATE_FULL) and 25 KiB per round workgroup (one per
 * 4096 nodes, at most 256 on MI355X): 256 MiB hold, for example, every graph
 * of up to 10^6 nodes and 32 * 10^6 entries.  A graph that does not fit
 * returns IPGC_ETOOBIG before any device work.  options->profile must be NULL
 * (IPGC_EINVAL): a profile needs events and a tick buffer.
 *
 * Every call on a GPU shares that GPU's array, which keeps the last call's
 * contents (the call clears what must start at zero).  The library serializes
 * its own calls per process and the call blocks until the result is complete,
 * so calls from one process never overlap; work that another party enqueues
 * into the same array would race.  Other arguments, errors and blocking are
 * as for ipgc_color_graph_ex.
 */
#define IPGC_NOALLOC_SCRATCH_BYTES (256ull << 20)
int ipgc_color_graph_noalloc(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int mode,
                             const ipgc_options *options, void *stream, int32_t *out_colors, int32_t *out_rounds,
                             ipgc_trace *trace);

/*
 * Color many graphs in one launch (the batched form of ipgc_color_graph).  The
 * graphs run together as one disjoint union; each one gets exactly the colors
 * and round count it gets alone.  One schedule decision is made per round for
 * the whole batch (topology-driven iff the batch's worklist exceeds H, by
 * default floor(6N/10) for N nodes in total).
 *
 * With IPGC_FLAG_PER_GRAPH each graph g decides for itself (Section IV applied to
 * each graph): its round r is topology-driven iff its own worklist, its nodes not
 * yet colored, holds more than H_g nodes, with H_g = floor(6 n_g / 10) by default
 * and floor(H n_g / N) for a threshold H > 0 given in the options (each graph the
 * same fraction of its nodes); TOPOLOGY and DATA give every graph that mode.  A
 * round in which graphs of both kinds have work runs each step as a pass over
 * the worklist for the data-driven graphs and a sweep over the nodes of the
 * topology-driven ones.  The results are those of the default form.  Limits: at
 * most 65536 graphs; not with IPGC_MODE_REBUILD (IPGC_EINVAL); the worklists take
 * twice the device memory of the default form.
 *
 * num_graphs     number of graphs G >= 0.
 * node_off       HOST, G + 1 entries: graph g has nodes [node_off[g], node_off[g+1]) of the
 *                packed color array; node_off[0] = 0.  Total nodes N = node_off[G] < 2^31 - 1.
 * edge_off       HOST, G + 1 entries: graph g's column indices are colidx_packed[edge_off[g] ..
 *                edge_off[g+1]); edge_off[0] = 0.  The total may exceed 2^31; each graph's
 *                count must not.
 * rowptr_packed  DEVICE, N + G int32 entries: graph g's own row pointers (n_g + 1 entries,
 *                starting at 0 and ending at its entry count) at rowptr_packed + node_off[g] + g.
 * colidx_packed  DEVICE, column indices local to each graph (in [0, n_g)).
 * out_colors_packed DEVICE, N int32 entries: graph g's colors at out_colors_packed + node_off[g].
 * out_rounds     HOST, G entries: each graph's round count (-1 for all on error).
 * trace          optional (NULL: none): per round of the whole batch, the size and degree sum of
 *                the union of the graphs' worklists and the kind of round run (with
 *                IPGC_FLAG_PER_GRAPH also topo_graphs: the graphs that ran it topology-driven).
 * Every local row pointer sequence is checked (starts at 0, non-decreasing, ends at the graph's
 * entry count) at every validation level; column ids are checked against their own graph's node
 * count unless validation is IPGC_VALIDATE_NONE.  IPGC_ETOOBIG if options->workgroups is so small
 * that a workgroup's worklist segment (N / workgroups + 1024 entries, twice that with
 * IPGC_FLAG_PER_GRAPH) would pass INT32_MAX.  Options, stream and blocking are as for
 * ipgc_color_graph_ex; the round limit is the batch's node count.
 */
int ipgc_color_graphs_batched(int64_t num_graphs, const int64_t *node_off, const int64_t *edge_off,
                              const int32_t *rowptr_packed, const int32_t *colidx_packed, int mode,
                              const ipgc_options *options, void *stream, int32_t *out_colors_packed,
                              int32_t *out_rounds, ipgc_trace *trace);

/*
 * Serving: a device-resident job server with continuous batching.
 *
 * A server owns a device arena sized once at creation: node slots, CSR entry
 * slots, byte-map bytes and job slots.  Submitted jobs wait in a FIFO queue
 * until the arena has room for them (memory admission); an admitted job's CSR,
 * color state, byte maps and rings stay resident until it completes.  Each
 * ipgc_server_step runs up to rounds_per_step rounds of IPGC over every
 * resident job at once (one cooperative launch, the jobs forming one disjoint
 * union), after retiring the jobs that completed and admitting queued jobs
 * that now fit.  Jobs that arrive while others are running join at the next
 * step, so their rounds overlap on the device with those of the jobs already
 * resident.  Every job gets exactly the colors and round count it gets alone
 * (the rules of ipgc_color_graph make each job's result independent of
 * everything else in the union).  The schedule of each round (topology-driven
 * iff the union's worklist exceeds H, by default floor(6 N / 10) for the N
 * resident nodes) changes only the time.
 *
 * A server is used from one thread at a time and runs on the device that was
 * current at creation.
 */
typedef struct ipgc_server ipgc_server;

typedef struct ipgc_server_config {
    int64_t node_capacity;    /* arena node slots; a job takes n + 1 */
    int64_t edge_capacity;    /* arena CSR entry slots; a job takes m */
    int32_t max_jobs;         /* jobs resident at once (job slots) */
    int32_t rounds_per_step;  /* rounds per ipgc_server_step (0: 8) */
    int32_t mode;             /* ipgc_mode of the rounds */
    int32_t reserved;         /* must be 0 */
    ipgc_options options;     /* threshold (0: floor(6N/10) over the resident nodes), light_max_degree,
                                 hub_min_degree, workgroups, IPGC_FLAG_LIGHT_PULL / _PUSH / _RACY;
                                 validate must not be IPGC_VALIDATE_NONE (every admitted job is
                                 checked); IPGC_FLAG_STEPPED and a profile are rejected */
} ipgc_server_config;

/* Outcome of a finished job. */
typedef struct ipgc_job_result {
    int64_t job_id;
    int32_t status;   /* IPGC_OK, or IPGC_EBADCSR if the job's CSR failed the checks */
    int32_t rounds;   /* the job's round count (-1 on error) */
} ipgc_job_result;

typedef struct ipgc_server_stats {
    int64_t steps;          /* ipgc_server_step calls that ran rounds */
    int64_t cancelled;      /* jobs cancelled before they finished */
    int64_t rounds;         /* rounds run (over the union) */
    int64_t submitted, admitted, completed;
    int64_t resident;       /* jobs resident now */
    int64_t queued;         /* jobs waiting for room */
    int64_t resident_nodes; /* nodes of the resident jobs */
    int64_t resident_edges; /* CSR entries of the resident jobs */
    int64_t peak_resident;  /* most jobs resident at once */
    int64_t arena_bytes;    /* device memory held by the server */
    int64_t units[IPGC_PROFILE_KINDS]; /* work units summed over all rounds (see ipgc_unit_name) */
} ipgc_server_stats;

/* Creates a server and allocates its arena on the current device.  Fails with
 * IPGC_ENOMEM if the arena does not fit, IPGC_EINVAL for a bad config. */
int ipgc_server_create(const ipgc_server_config *config, ipgc_server **out);

/*
 * Queues a job.  rowptr (n + 1 int32) and colidx (m int32, ids in [0, n)) are
 * HOST pointers in the CSR format of ipgc_color_graph; out_colors is a HOST
 * array of n int32 that receives the colors when the job completes.  All three
 * must stay valid until ipgc_server_poll reports the job.  IPGC_ETOOBIG if the
 * job can never fit the arena; IPGC_EINVAL for negative sizes or null
 * pointers.  job_id receives the job's id (ids count up from 0).
 */
int ipgc_server_submit(ipgc_server *server, const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t m,
                       int32_t *out_colors, int64_t *job_id);

/* One step: retire completed jobs (their colors are copied to out_colors),
 * admit queued jobs in FIFO order while they fit, then run up to
 * rounds_per_step rounds over the resident jobs.  Blocks until the rounds are
 * done.  Does nothing if no job is resident or queued. */
int ipgc_server_step(ipgc_server *server);

/* Results of the jobs finished since the last poll, oldest first: up to
 * capacity entries go to results, their number to count.  A job finishes
 * during the step after the one in which its last node committed, or at once
 * if it failed its checks or has no nodes. */
int ipgc_server_poll(ipgc_server *server, ipgc_job_result *results, int64_t capacity, int64_t *count);

int ipgc_server_stats_get(const ipgc_server *server, ipgc_server_stats *stats);

/*
 * Runs steps until job job_id has finished, then takes its result out of the
 * list of finished jobs (so ipgc_server_poll will not report it) and stores it
 * in *result.  The job's out_colors are filled if its status is IPGC_OK.  Jobs
 * that finish on the way stay in the list for ipgc_server_poll.  Returns
 * IPGC_EINVAL if no job with that id is queued, resident or finished and not
 * yet reported; errors of ipgc_server_step are returned as they occur.
 */
int ipgc_server_wait(ipgc_server *server, int64_t job_id, ipgc_job_result *result);

/*
 * Cancels a job that has not finished.  A queued job is dropped; a job whose
 * upload is under way is dropped once the upload has ended (the call waits for
 * it); a resident job leaves the union before the next round, and its arena
 * ranges are freed.  Its out_colors are never written, and it is reported
 * (ipgc_server_poll / ipgc_server_wait) with status IPGC_ECANCELED and rounds
 * -1.  Every other job's result is unchanged: jobs in the union never read one
 * another's state.  Returns IPGC_EINVAL if the job has already finished or no
 * such job exists.
 */
int ipgc_server_cancel(ipgc_server *server, int64_t job_id);

/* Frees the arena.  Queued and resident jobs are dropped. */
void ipgc_server_destroy(ipgc_server *server);

/*
 * Breadth-first search under the same keep-the-worklist hybrid schedule (the
 * paper's driver applied to another worklist algorithm, as its conclusion
 * proposes).  Level L expands the nodes at distance L, either by a sweep over
 * all nodes (topology-driven, iff the frontier holds more than H nodes; by
 * default H = floor(6n/10)) or by walking the worklist (data-driven); both
 * kinds push every newly reached node onto the next worklist.
 *
 * csr_rowptr, csr_colidx  DEVICE, the CSR of ipgc_color_graph (read only).
 * source      the start node, in [0, n).
 * mode        IPGC_MODE_TOPOLOGY, _DATA or _HYBRID (REBUILD is rejected).
 * options     threshold, workgroups and validate are used (NULL: defaults); flags must be 0.
 * out_dist    DEVICE, n int32: hops from the source, -1 if unreachable.
 * out_levels  HOST: the number of non-empty frontiers (the largest finite distance + 1).
 * trace       optional: the frontier size of every level and its kind.
 * Blocks until done; returns the ipgc_color_graph error codes.
 */
int ipgc_bfs(const int32_t *csr_rowptr, const int32_t *csr_colidx, int64_t n, int64_t m, int64_t source, int mode,
             const ipgc_options *options, void *stream, int32_t *out_dist, int32_t *out_levels, ipgc_trace *trace);

/*
 * Worklist push micro-benchmark (Section III, Listings 1 and 2): starting from
 * a worklist of all n node ids, iteration i deactivates ids [count*i,
 * count*(i+1)) and pushes the rest into the next worklist, iterating over the
 * worklist (nowl = 0: Push_WL) or over every id (nowl = 1: Push_NoWL), until
 * the worklist is empty.  atomic = 0 pushes with per-workgroup segments and no
 * global atomic (as the coloring kernels do); atomic = 1 fills one global
 * worklist with one atomicAdd per wavefront.  One kernel launch per
 * iteration: the launch boundary separates iterations, and the first
 * workgroup of each launch stamps the device clock, so an iteration's time
 * includes its launch.  HOST arrays of `capacity` entries (at least
 * ceil(n/count) + 2) receive the device wall clock at the start of every
 * iteration plus one at the end (ticks) and the worklist size at the start of
 * every iteration (sizes); iterations receives the number of non-empty
 * iterations and tick_khz the rate of the clock.  Runs on the current device
 * and blocks until done.  The time per iteration i is
 * (ticks[i+1] - ticks[i]) / tick_khz milliseconds.
 */
int ipgc_push_microbench(int64_t n, int32_t count, int32_t nowl, int32_t atomic, uint64_t *ticks, int32_t *sizes,
                         int64_t capacity, int64_t *iterations, int64_t *tick_khz);

/* Message for the last failing call on this thread ("" if none).  Valid until
 * the next call on the same thread. */
const char *ipgc_last_error(void);

/* Name of profile kernel kind k ("" past the last kind). */
const char *ipgc_kernel_name(int kind);

/* Name of profile work unit kind k ("" past the last kind). */
const char *ipgc_unit_name(int kind);

/* ABI version: (major << 16) | minor. */
int ipgc_version(void);

/* Releases the cached per-device workspaces (of the coloring and BFS entry
 * points).  Optional; safe to call anytime no other call is in flight. */
void ipgc_release_workspaces(void);

/*
 * Device memory hook.  By default the library takes device memory with
 * hipMalloc and returns it with hipFree: its cached workspaces (which only
 * grow) and the arena of each server (sized at ipgc_server_create).  A caller
 * that manages device memory itself (a framework's caching allocator, a
 * memory budget, a test that injects failures) installs alloc/free here:
 * alloc(bytes, device, user) returns a device pointer on `device` aligned to
 * at least 256 bytes, or NULL, which the library reports as IPGC_ENOMEM after
 * freeing what the failing call had taken; free(ptr, bytes, device, user)
 * takes back a pointer that alloc returned (with the same size).  Memory is
 * always returned to the hook pair that gave it, even after the hook has been
 * replaced.  Both NULL restore hipMalloc/hipFree.  IPGC_EINVAL if exactly one
 * of them is NULL.  Install the hook when no other library call is in flight.
 */
typedef void *(*ipgc_alloc_fn)(uint64_t bytes, int device, void *user);
typedef void (*ipgc_free_fn)(void *ptr, uint64_t bytes, int device, void *user);
int ipgc_set_allocator(ipgc_alloc_fn alloc, ipgc_free_fn free_fn, void *user);

#ifdef __cplusplus
}
#endif

#endif /* IPGC_H */
