/*
 * CPU oracle for breadth-first search -- TEST INFRASTRUCTURE ONLY.
 *
 * The keep-the-worklist hybrid of Rai, M P, Pai, "A Hybrid Graph Coloring
 * Algorithm for GPUs" (arXiv 1912.01478) is a driver for any worklist
 * algorithm; its conclusion names other algorithms as the next step.  The GPU
 * library applies it to level-synchronous BFS, whose result is defined without
 * reference to any schedule: dist[v] is the number of edges on a shortest path
 * from the source to v, or -1 if v is unreachable.  This file computes that
 * definition with a FIFO queue, and records the size of every frontier (the
 * nodes at distance L, for L = 0, 1, ...) so that the GPU's worklist trace can
 * be compared.  It shares no code with the HIP library.
 */
#include <stdint.h>
#include <stdlib.h>

/*
 * dist (n entries) receives the distances; sizes (capacity `cap`) the number of
 * nodes at each distance; *levels the number of non-empty frontiers (the
 * largest finite distance + 1).  Returns 0, -1 for bad arguments, -2 if memory
 * runs out, -3 for a column id outside [0, n).
 */
int ipgc_oracle_bfs(const int32_t *rowptr, const int32_t *colidx, int64_t n, int64_t source, int32_t *dist,
                    int64_t *sizes, int64_t cap, int32_t *levels) {
    if (n < 0 || !rowptr || !dist || !levels || (n > 0 && (source < 0 || source >= n))) return -1;
    *levels = 0;
    if (n == 0) return 0;
    int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!queue) return -2;
    for (int64_t v = 0; v < n; ++v) dist[v] = -1;
    int64_t head = 0, tail = 0;
    dist[source] = 0;
    queue[tail++] = (int32_t)source;
    while (head < tail) {
        const int32_t v = queue[head++];
        for (int64_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
            const int32_t u = colidx[e];
            if (u < 0 || u >= n) {
                free(queue);
                return -3;
            }
            if (dist[u] < 0) {
                dist[u] = dist[v] + 1;
                queue[tail++] = u;
            }
        }
    }
    /* frontier sizes: nodes per distance, in BFS order the distances are non-decreasing */
    for (int64_t i = 0; i < tail; ++i) {
        const int32_t d = dist[queue[i]];
        if (d + 1 > *levels) *levels = d + 1;
        if (d < cap) sizes[d] += 1;
    }
    free(queue);
    return 0;
}
