/*
 * CPU oracle for IPGC (Iterative Parallel Graph Coloring) -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the plain, slow, single-threaded definition of what the GPU
 * coloring library must compute.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never does.  It
 * shares no code, header, table or constant with the HIP library.
 *
 * Method: Rai, M P, Pai, "A Hybrid Graph Coloring Algorithm for GPUs"
 * (arXiv 1912.01478), Section II-C (IPGC) with its footnote on mex, and
 * Section IV (the hybrid driver that picks a topology-driven or data-driven
 * round from the worklist size against a threshold H).  The schedule never
 * changes the result: Section V states that all versions produce the same
 * colors because they run the same coloring algorithm, so the oracle computes
 * one result and only labels each round with the kind the hybrid driver would
 * pick for it.
 *
 * Readings where the paper is silent or loose (each one is listed with its
 * justification in the design notes of the repository):
 *   R1 colors are 1-based; 0 means "uncolored" (Section II-C sets every node
 *      to 0 = uncolored initially), so a node takes the smallest c >= 1 that
 *      no committed neighbour holds, i.e. mex(F u {0}).
 *   R2 only committed colors forbid: nodes uncolored after a conflict hold 0.
 *   R3 synchronous rounds: every assignment in a round reads the colors as they
 *      stood at the start of the round, and every conflict test reads the
 *      tentative colors as they stood after the whole assignment step.
 *   R4 a conflict on edge (u, v) with u < v uncolors v and lets u keep its
 *      color (the paper says one endpoint is removed but not which); v loses
 *      even when u also loses to a smaller neighbour.
 *   R5 the round count is the number of assign+conflict iterations run until
 *      the worklist is empty, the last one included.
 *   R6 round kind: topology-driven iff |WL| > H (default H = floor(6n/10),
 *      Section IV reports H around 60% of the node count); data-driven
 *      otherwise.  This labels rounds only; colors do not depend on it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORACLE_OK = 0, ORACLE_EINVAL = -1, ORACLE_ENOMEM = -2, ORACLE_EBADCSR = -3 };

/*
 * mex over the committed colors of v's neighbours, 1-based (footnote on mex in
 * Section II-C, reading R1).  `seen` has room for deg+2 flags; a node of degree
 * d can only see d colors, so the answer lies in [1, d+1].
 */
static int32_t first_free_color(const int32_t *rowptr, const int32_t *colidx, const int32_t *col,
                                int64_t v, unsigned char *seen) {
    int64_t d = (int64_t)rowptr[v + 1] - rowptr[v];
    memset(seen, 0, (size_t)(d + 2));
    for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
        int32_t c = col[colidx[e]];
        if (c >= 1 && c <= d + 1) seen[c] = 1;
    }
    int32_t c = 1;
    while (seen[c]) ++c;
    return c;
}

/*
 * Color a graph with synchronous IPGC (Section II-C, readings R1-R5).
 *
 * rowptr[n+1], colidx[m]: symmetric CSR in host memory.  Self-loops are not
 *   expected; one would change nothing, since a node is uncolored while it is
 *   active (so it forbids nothing to itself) and u < v is strict.
 * threshold: H for the round labels (R6); negative selects floor(6n/10).
 * col_out[n]: final colors (1-based).
 * rounds_out: number of rounds.
 * commit_round[n] (nullable): the round in which each node kept its color.
 * trace_cap and trace_* (nullable): per round r < trace_cap, the worklist size
 *   |WL_r|, the degree sum of the worklist D_r, and 1 if the round is
 *   topology-driven under H.
 * max_rounds: stop after this many rounds even if the worklist is not empty
 *   (<= 0: no limit).  A stopped run leaves some nodes at color 0; it exists
 *   only to time a bounded sample of a large workload.
 * Returns 0, or a negative error code.
 */
int ipgc_oracle_color(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t threshold,
                      int32_t *col_out, int32_t *rounds_out, int32_t *commit_round, int64_t trace_cap,
                      int64_t *trace_wl, int64_t *trace_deg, int32_t *trace_topo, int64_t max_rounds) {
    if (n < 0 || !rounds_out || (n > 0 && (!rowptr || !colidx || !col_out))) return ORACLE_EINVAL;
    *rounds_out = 0;
    if (n == 0) return ORACLE_OK;
    if (rowptr[0] != 0) return ORACLE_EBADCSR;
    int64_t maxdeg = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t d = (int64_t)rowptr[v + 1] - rowptr[v];
        if (d < 0) return ORACLE_EBADCSR;
        if (d > maxdeg) maxdeg = d;
    }
    for (int64_t e = 0; e < rowptr[n]; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return ORACLE_EBADCSR;
    const int64_t H = threshold < 0 ? (6 * n) / 10 : threshold;

    int32_t *col = col_out;
    int32_t *tent = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *wl = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    unsigned char *in_wl = (unsigned char *)malloc((size_t)n);
    unsigned char *lose = (unsigned char *)malloc((size_t)n);
    unsigned char *seen = (unsigned char *)malloc((size_t)(maxdeg + 2));
    if (!tent || !wl || !in_wl || !lose || !seen) {
        free(tent); free(wl); free(in_wl); free(lose); free(seen);
        return ORACLE_ENOMEM;
    }

    /* Initial state (Section II-C): every node has color 0, i.e. uncolored and
     * conflicting, and the worklist holds every node. */
    for (int64_t v = 0; v < n; ++v) {
        col[v] = 0;
        tent[v] = 0;
        wl[v] = v;
        in_wl[v] = 1;
        if (commit_round) commit_round[v] = 0;
    }
    int64_t wl_len = n;
    int32_t r = 0;

    /* The loop runs while the worklist is non-empty (Section II-C: the
     * algorithm ends when the worklist is empty). */
    while (wl_len > 0 && (max_rounds <= 0 || r < max_rounds)) {
        ++r;
        if (r - 1 < trace_cap) {
            int64_t dsum = 0;
            for (int64_t i = 0; i < wl_len; ++i) dsum += (int64_t)rowptr[wl[i] + 1] - rowptr[wl[i]];
            if (trace_wl) trace_wl[r - 1] = wl_len;
            if (trace_deg) trace_deg[r - 1] = dsum;
            if (trace_topo) trace_topo[r - 1] = wl_len > H ? 1 : 0;
        }

        /* Step 1: every uncolored node takes a color unused by its
         * neighbours, all from the same snapshot of `col` (R3). */
        for (int64_t i = 0; i < wl_len; ++i) {
            int64_t v = wl[i];
            tent[v] = first_free_color(rowptr, colidx, col, v, seen);
        }

        /* Step 2: where an edge joins two nodes of the worklist holding the
         * same tentative color, the larger id is uncolored (R4).  Evaluated
         * on the full set of tentative colors from step 1 (R3). */
        for (int64_t i = 0; i < wl_len; ++i) {
            int64_t v = wl[i];
            lose[v] = 0;
            for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int64_t u = colidx[e];
                if (u < v && in_wl[u] && tent[u] == tent[v]) { lose[v] = 1; break; }
            }
        }

        /* Nodes without a conflict keep their color and leave the worklist;
         * the others stay uncolored (R2) and form the next worklist, which
         * keeps ascending id order. */
        int64_t next = 0;
        for (int64_t i = 0; i < wl_len; ++i) {
            int64_t v = wl[i];
            if (lose[v]) {
                wl[next++] = v;
            } else {
                col[v] = tent[v];
                in_wl[v] = 0;
                if (commit_round) commit_round[v] = r;
            }
        }
        wl_len = next;
    }
    *rounds_out = r;
    free(tent); free(wl); free(in_wl); free(lose); free(seen);
    return ORACLE_OK;
}

/* The assignment rule on its own, for the footnote pin: the color node v
 * would take given the committed colors `col` of every node (footnote on mex
 * in Section II-C, reading R1).  Returns -1 on bad arguments. */
int32_t ipgc_oracle_first_free_color(const int32_t *rowptr, const int32_t *colidx, int64_t n,
                                     const int32_t *col, int64_t v) {
    if (!rowptr || !colidx || !col || v < 0 || v >= n) return -1;
    int64_t d = (int64_t)rowptr[v + 1] - rowptr[v];
    unsigned char *seen = (unsigned char *)malloc((size_t)(d + 2));
    if (!seen) return -1;
    int32_t c = first_free_color(rowptr, colidx, col, v, seen);
    free(seen);
    return c;
}
