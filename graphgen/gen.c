/*
 * Seeded synthetic graph generators (host C, no GPU, no coloring arithmetic).
 *
 * These produce the inputs that both the CPU oracle and the HIP coloring path
 * consume; they contain nothing of the coloring method itself.  Every random
 * draw comes from a counter-based stream: value(key, i) is output number i of
 * the SplitMix64 generator (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014) whose state starts at `key`.  Because each
 * draw is a pure function of (key, i), results do not depend on thread count.
 *
 * Output format everywhere: canonical symmetric CSR with int32 row pointers and
 * column indices, rows sorted ascending, no self-loops, no duplicate entries.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

/* Output number `ctr` (0-based) of SplitMix64 seeded with `key`. */
static inline uint64_t draw(uint64_t key, uint64_t ctr) {
    uint64_t z = key + (ctr + 1) * GOLDEN;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gg_draw(uint64_t key, uint64_t ctr) { return draw(key, ctr); }

/* Uniform double in [0,1) from the top 53 bits of a draw. */
static inline double unit_double(uint64_t r) { return (double)(int64_t)(r >> 11) * (1.0 / 9007199254740992.0); }

/* Stream key for (a, b), e.g. (config id, graph index). */
uint64_t gg_key(uint64_t a, uint64_t b) { return draw(draw(a, 0x5eed) ^ b, 0x5eed); }

/* One R-MAT sample: draws (i*scale + l) for levels l = 0..scale-1; each level picks a quadrant
 * with probabilities (a, b, c, 1-a-b-c) and appends one bit to each endpoint. */
static inline void rmat_sample(int32_t scale, double a, double ab, double abc, uint64_t key, uint64_t i,
                               uint64_t *pu, uint64_t *pv) {
    uint64_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
        double r = unit_double(draw(key, i * (uint64_t)scale + (uint64_t)l));
        /* quadrant bits without branches (the comparisons are random, so branches mispredict) */
        const uint64_t ge_a = r >= a, ge_ab = r >= ab, ge_abc = r >= abc;
        const uint64_t bu = ge_ab, bv = (ge_a & (ge_ab ^ 1)) | ge_abc;
        u = (u << 1) | bu;
        v = (v << 1) | bv;
    }
    *pu = u;
    *pv = v;
}

/*
 * R-MAT edge samples on 2^scale ids.  Sample index i is a pure function of (key, i).  When
 * `nmax` is below 2^scale, samples with an endpoint >= nmax are rejected and sampling continues
 * with the next sample index until `want` samples are accepted (accepted samples keep index
 * order).  Returns the number of sample indices consumed.
 */
int64_t gg_rmat(int32_t scale, int64_t nmax, int64_t want, double a, double b, double c, uint64_t key,
                int32_t *src, int32_t *dst) {
    const double ab = a + b, abc = a + b + c;
    int64_t chunk = 2 * want + 4096; /* the chunk size changes only the work wasted past the last sample */
    if (chunk > (1 << 20)) chunk = 1 << 20;
    uint64_t *tu = (uint64_t *)malloc(sizeof(uint64_t) * chunk);
    uint64_t *tv = (uint64_t *)malloc(sizeof(uint64_t) * chunk);
    if (!tu || !tv) { free(tu); free(tv); return -1; }
    int64_t got = 0, i0 = 0;
    while (got < want) {
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < chunk; ++j) rmat_sample(scale, a, ab, abc, key, (uint64_t)(i0 + j), &tu[j], &tv[j]);
        int64_t j = 0;
        for (; j < chunk && got < want; ++j) {
            if ((int64_t)tu[j] >= nmax || (int64_t)tv[j] >= nmax) continue;
            src[got] = (int32_t)tu[j];
            dst[got] = (int32_t)tv[j];
            ++got;
        }
        i0 += j;
    }
    free(tu); free(tv);
    return i0;
}

/* Uniform node pairs (u, v) with u != v on n nodes, draws starting at counter ctr0. */
void gg_uniform_pairs(int64_t n, int64_t count, uint64_t key, uint64_t ctr0, int32_t *src, int32_t *dst) {
    for (int64_t i = 0; i < count; ++i) {
        uint64_t ctr = ctr0 + 2 * (uint64_t)i;
        for (;;) {
            uint64_t u = draw(key, ctr) % (uint64_t)n;
            uint64_t v = draw(key, ctr + 1) % (uint64_t)n;
            if (u != v) { src[i] = (int32_t)u; dst[i] = (int32_t)v; break; }
            ctr += 0x100000000ULL; /* retry on a disjoint counter range */
        }
    }
}

/* Apply a node relabelling: x -> perm[x] in place. */
void gg_relabel(int64_t count, const int32_t *perm, int32_t *x) {
    for (int64_t i = 0; i < count; ++i) x[i] = perm[x[i]];
}

/* Random permutation of [0, n) (Fisher-Yates driven by the draw stream). */
void gg_permutation(int64_t n, uint64_t key, int32_t *perm) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        uint64_t j = draw(key, (uint64_t)i) % (uint64_t)(i + 1);
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Canonical symmetric CSR from `np` undirected pairs on n nodes: self-loops are
 * dropped, both directions are added, rows are sorted and duplicates removed.
 * rowptr has n+1 entries; colidx must hold 2*np entries.  Returns m (the
 * number of CSR entries written), or -1 on allocation failure.  The result is
 * independent of thread count and of the order of the pairs.
 */
int64_t gg_build_csr(int64_t n, int64_t np, const int32_t *src, const int32_t *dst, int32_t *rowptr, int32_t *colidx) {
    int64_t *cur = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * np + 1));
    if (!cur || !cnt || !tmp) { free(cur); free(cnt); free(tmp); return -1; }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
        if (src[i] == dst[i]) continue;
#pragma omp atomic
        cur[src[i] + 1]++;
#pragma omp atomic
        cur[dst[i] + 1]++;
    }
    for (int64_t v = 0; v < n; ++v) cur[v + 1] += cur[v];
    int64_t *beg = cnt; /* reuse: row start of the unsorted layout */
    memcpy(beg, cur, sizeof(int64_t) * ((size_t)n + 1));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < np; ++i) {
        if (src[i] == dst[i]) continue;
        int64_t p, q;
#pragma omp atomic capture
        p = cur[src[i]]++;
#pragma omp atomic capture
        q = cur[dst[i]]++;
        tmp[p] = dst[i];
        tmp[q] = src[i];
    }
    /* cur[v] now equals beg[v+1]; sort and deduplicate each row in place, keep new lengths in cur */
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v) {
        int64_t b = beg[v], e = beg[v + 1];
        if (e - b > 1) qsort(tmp + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t w = b;
        for (int64_t i = b; i < e; ++i)
            if (i == b || tmp[i] != tmp[i - 1]) tmp[w++] = tmp[i];
        cur[v] = w - b;
    }
    int64_t m = 0;
    rowptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) { m += cur[v]; rowptr[v + 1] = (int32_t)m; }
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t v = 0; v < n; ++v)
        memmove(colidx + rowptr[v], tmp + beg[v], sizeof(int32_t) * (size_t)cur[v]);
    free(cur); free(cnt); free(tmp);
    return m;
}

/* n uniform points in [0,1)^2: x from draw 2i, y from draw 2i+1. */
void gg_points(int64_t n, uint64_t key, double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        x[i] = unit_double(draw(key, 2 * (uint64_t)i));
        y[i] = unit_double(draw(key, 2 * (uint64_t)i + 1));
    }
}

typedef struct { double x; int32_t i; } xkey;
static int cmp_xkey(const void *a, const void *b) {
    const xkey *p = (const xkey *)a, *q = (const xkey *)b;
    if (p->x != q->x) return (p->x > q->x) - (p->x < q->x);
    return (p->i > q->i) - (p->i < q->i);
}

/* Locality order of points: `strips` horizontal strips by y, x-sorted inside each strip.
 * order[new_id] = old point index. */
int gg_strip_order(int64_t n, const double *x, const double *y, int64_t strips, int32_t *order) {
    int64_t *start = (int64_t *)calloc((size_t)strips + 1, sizeof(int64_t));
    xkey *tmp = (xkey *)malloc(sizeof(xkey) * (size_t)(n + 1));
    if (!start || !tmp) { free(start); free(tmp); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = (int64_t)(y[i] * (double)strips);
        if (s >= strips) s = strips - 1;
        start[s + 1]++;
    }
    for (int64_t s = 0; s < strips; ++s) start[s + 1] += start[s];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)strips);
    if (!fill) { free(start); free(tmp); return -1; }
    memcpy(fill, start, sizeof(int64_t) * (size_t)strips);
    for (int64_t i = 0; i < n; ++i) {
        int64_t s = (int64_t)(y[i] * (double)strips);
        if (s >= strips) s = strips - 1;
        int64_t p = fill[s]++;
        tmp[p].x = x[i];
        tmp[p].i = (int32_t)i;
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t s = 0; s < strips; ++s)
        qsort(tmp + start[s], (size_t)(start[s + 1] - start[s]), sizeof(xkey), cmp_xkey);
    for (int64_t i = 0; i < n; ++i) order[i] = tmp[i].i;
    free(fill); free(start); free(tmp);
    return 0;
}

/*
 * k-nearest-neighbour links on points in the unit square, k[i] in [1, 8] per
 * point.  Neighbours are ordered by (squared distance, id).  Point i writes its
 * k[i] links as pairs (i, j) at slots [8*i, 8*i + k[i]); unused slots get
 * (i, i), which gg_build_csr drops as self-loops.  Grid search with a uniform
 * cell size; the search stops once the k-th best distance is no larger than
 * the distance to the unsearched region.
 */
int gg_knn(int64_t n, const double *x, const double *y, const int8_t *k, int32_t *src, int32_t *dst) {
    if (n <= 0) return 0;
    int64_t G = (int64_t)floor(sqrt((double)n / 2.0));
    if (G < 1) G = 1;
    int64_t ncell = G * G;
    int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *cellof = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!start || !order || !cellof) { free(start); free(order); free(cellof); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        int64_t cx = (int64_t)(x[i] * (double)G), cy = (int64_t)(y[i] * (double)G);
        if (cx >= G) cx = G - 1;
        if (cy >= G) cy = G - 1;
        cellof[i] = (int32_t)(cy * G + cx);
        start[cellof[i] + 1]++;
    }
    for (int64_t c = 0; c < ncell; ++c) start[c + 1] += start[c];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncell);
        if (!fill) { free(start); free(order); free(cellof); return -1; }
        memcpy(fill, start, sizeof(int64_t) * (size_t)ncell);
        for (int64_t i = 0; i < n; ++i) order[fill[cellof[i]]++] = (int32_t)i;
        free(fill);
    }
    const double h = 1.0 / (double)G;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
        int ki = k[i];
        double bd[8];
        int32_t bj[8];
        int nb = 0;
        int64_t cx = cellof[i] % G, cy = cellof[i] / G;
        for (int64_t R = 0;; ++R) {
            int64_t x0 = cx - R, x1 = cx + R, y0 = cy - R, y1 = cy + R;
            for (int64_t gy = y0; gy <= y1; ++gy) {
                if (gy < 0 || gy >= G) continue;
                for (int64_t gx = x0; gx <= x1; ++gx) {
                    if (gx < 0 || gx >= G) continue;
                    if (R > 0 && gy != y0 && gy != y1 && gx != x0 && gx != x1) continue; /* ring only */
                    int64_t c = gy * G + gx;
                    for (int64_t p = start[c]; p < start[c + 1]; ++p) {
                        int32_t j = order[p];
                        if (j == (int32_t)i) continue;
                        double dx = x[j] - x[i], dy = y[j] - y[i];
                        double dd = dx * dx + dy * dy;
                        if (nb == ki && (dd > bd[nb - 1] || (dd == bd[nb - 1] && j > bj[nb - 1]))) continue;
                        int q = nb < ki ? nb++ : nb - 1;
                        while (q > 0 && (bd[q - 1] > dd || (bd[q - 1] == dd && bj[q - 1] > j))) {
                            bd[q] = bd[q - 1]; bj[q] = bj[q - 1]; --q;
                        }
                        bd[q] = dd; bj[q] = j;
                    }
                }
            }
            /* distance from the point to the nearest unsearched cell (sides past the border are never searched) */
            double lim = 1e300;
            if (x0 - 1 >= 0) { double t = x[i] - (double)x0 * h; if (t < lim) lim = t; }
            if (x1 + 1 < G) { double t = (double)(x1 + 1) * h - x[i]; if (t < lim) lim = t; }
            if (y0 - 1 >= 0) { double t = y[i] - (double)y0 * h; if (t < lim) lim = t; }
            if (y1 + 1 < G) { double t = (double)(y1 + 1) * h - y[i]; if (t < lim) lim = t; }
            int all_searched = (x0 <= 0 && y0 <= 0 && x1 >= G - 1 && y1 >= G - 1);
            if (all_searched) break;
            if (nb == ki && bd[nb - 1] <= lim * lim) break;
        }
        for (int q = 0; q < 8; ++q) {
            src[8 * i + q] = (int32_t)i;
            dst[8 * i + q] = q < nb ? bj[q] : (int32_t)i;
        }
    }
    free(start); free(order); free(cellof);
    return 0;
}

/* Pair index i -> (u, v): the uniform pair gg_uniform_pairs writes for counter 2i. */
static inline void pair_at(int64_t n, uint64_t key, uint64_t i, uint64_t *pu, uint64_t *pv) {
    uint64_t ctr = 2 * i;
    for (;;) {
        uint64_t u = draw(key, ctr) % (uint64_t)n;
        uint64_t v = draw(key, ctr + 1) % (uint64_t)n;
        if (u != v) { *pu = u; *pv = v; return; }
        ctr += 0x100000000ULL;
    }
}

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/*
 * G(n, M): the first M distinct unordered pairs of the uniform pair stream (pair i drawn at
 * counter 2i, self-pairs redrawn), in draw order, via an open-addressing set of the pair keys.
 * M must not exceed n(n-1)/2.  Returns the number of pair indices consumed, or -1.
 */
int64_t gg_er_pairs(int64_t n, int64_t M, uint64_t key, int32_t *src, int32_t *dst) {
    if (M <= 0) return 0;
    uint64_t cap = 64;
    while (cap < 2 * (uint64_t)M) cap <<= 1;
    uint64_t *tab = (uint64_t *)calloc(cap, sizeof(uint64_t));
    if (!tab) return -1;
    /* pairs are drawn PF ahead of their insertion so that their table slots can be prefetched */
    enum { PF = 16 };
    uint64_t ku[PF], kv[PF], kk[PF], kh[PF];
    for (int j = 0; j < PF; ++j) {
        pair_at(n, key, (uint64_t)j, &ku[j], &kv[j]);
        const uint64_t lo = ku[j] < kv[j] ? ku[j] : kv[j], hi = ku[j] < kv[j] ? kv[j] : ku[j];
        kk[j] = lo * (uint64_t)n + hi + 1; /* 0 marks an empty slot */
        kh[j] = mix64(kk[j]) & (cap - 1);
        __builtin_prefetch(&tab[kh[j]], 1);
    }
    int64_t got = 0;
    uint64_t i = 0;
    for (; got < M; ++i) {
        const int j = (int)(i % PF);
        const uint64_t u = ku[j], v = kv[j], k = kk[j];
        uint64_t h = kh[j];
        /* refill slot j with pair i + PF */
        pair_at(n, key, i + PF, &ku[j], &kv[j]);
        {
            const uint64_t lo = ku[j] < kv[j] ? ku[j] : kv[j], hi = ku[j] < kv[j] ? kv[j] : ku[j];
            kk[j] = lo * (uint64_t)n + hi + 1;
            kh[j] = mix64(kk[j]) & (cap - 1);
            __builtin_prefetch(&tab[kh[j]], 1);
        }
        while (tab[h] && tab[h] != k) h = (h + 1) & (cap - 1);
        if (tab[h]) continue;
        tab[h] = k;
        src[got] = (int32_t)u;
        dst[got] = (int32_t)v;
        ++got;
    }
    free(tab);
    return (int64_t)i;
}

static void sort_row(int32_t *x, int64_t len) {
    if (len > 48) { qsort(x, (size_t)len, sizeof(int32_t), cmp_i32); return; }
    for (int64_t i = 1; i < len; ++i) {
        const int32_t t = x[i];
        int64_t j = i - 1;
        while (j >= 0 && x[j] > t) { x[j + 1] = x[j]; --j; }
        x[j + 1] = t;
    }
}

/* The canonical CSR of gg_build_csr, built by the calling thread alone (for one graph per
 * thread).  colidx must hold 2*np entries; it doubles as the scatter buffer. */
static int64_t build_csr_serial(int64_t n, int64_t np, const int32_t *src, const int32_t *dst, int32_t *rowptr,
                                int32_t *colidx) {
    int64_t *beg = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
    if (!beg) return -1;
    for (int64_t i = 0; i < np; ++i) {
        if (src[i] == dst[i]) continue;
        beg[src[i] + 2]++;
        beg[dst[i] + 2]++;
    }
    for (int64_t v = 0; v < n; ++v) beg[v + 2] += beg[v + 1];
    /* beg[v + 1] is now row v's start; use it as the fill cursor, after which it is row v's end */
    for (int64_t i = 0; i < np; ++i) {
        if (src[i] == dst[i]) continue;
        colidx[beg[src[i] + 1]++] = dst[i];
        colidx[beg[dst[i] + 1]++] = src[i];
    }
    int64_t w = 0, b = 0;
    rowptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        const int64_t e = beg[v + 1];
        sort_row(colidx + b, e - b);
        for (int64_t i = b; i < e; ++i)
            if (i == b || colidx[i] != colidx[i - 1]) colidx[w++] = colidx[i];
        rowptr[v + 1] = (int32_t)w;
        b = e;
    }
    free(beg);
    return w;
}

/* Whole G(n, M) graph as canonical CSR; colidx must hold 2M entries.  Returns m or -1. */
int64_t gg_er_csr(int64_t n, int64_t M, uint64_t key, int32_t *rowptr, int32_t *colidx) {
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)(M + 1));
    int64_t m = -1;
    if (s && d && gg_er_pairs(n, M, key, s, d) >= 0) m = build_csr_serial(n, M, s, d, rowptr, colidx);
    free(s); free(d);
    return m;
}

/* Whole R-MAT graph (samples, optional seeded permutation, canonical CSR) on n <= 2^scale nodes;
 * colidx must hold 2 * edge_factor * n entries.  Returns m or -1. */
int64_t gg_rmat_csr(int32_t scale, int64_t n, int64_t edge_factor, double a, double b, double c, uint64_t key,
                    int permute, int32_t *rowptr, int32_t *colidx) {
    const int64_t want = edge_factor * n;
    int32_t *s = (int32_t *)malloc(sizeof(int32_t) * (size_t)(want + 1));
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)(want + 1));
    int32_t *perm = permute ? (int32_t *)malloc(sizeof(int32_t) * (size_t)(n + 1)) : NULL;
    int64_t m = -1;
    if (s && d && (perm || !permute) && gg_rmat(scale, n, want, a, b, c, key, s, d) >= 0) {
        if (permute) {
            gg_permutation(n, draw(key, 0xFFFFFFFFFFFFULL), perm);
            gg_relabel(want, perm, s);
            gg_relabel(want, perm, d);
        }
        m = build_csr_serial(n, want, s, d, rowptr, colidx);
    }
    free(s); free(d); free(perm);
    return m;
}

/*
 * Graphs order[0 .. count-1] of a batch, generated in parallel (one graph per thread, in the
 * given order; pass larger graphs first).  Graph g: kind[g] 0 = G(n, M) with M = param[g], 1 =
 * R-MAT with edge factor param[g] on scale[g]; stream key key[g].  Its local row pointers go to
 * rowptr_packed + node_off[g] + g and its column ids to colidx_packed + cap_off[g] (room for
 * cap_off[g+1] - cap_off[g] entries); m_out[g] receives its entry count.  Returns 0, or -1 - g
 * for a failed graph g.
 */
int64_t gg_batch(int64_t count, const int32_t *kind, const int32_t *scale, const int64_t *param, const uint64_t *key,
                 const int64_t *node_off, const int64_t *cap_off, const int64_t *order, int32_t *rowptr_packed,
                 int32_t *colidx_packed, int64_t *m_out) {
    int64_t fail = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = 0; j < count; ++j) {
        const int64_t g = order[j];
        const int64_t n = node_off[g + 1] - node_off[g];
        int32_t *rp = rowptr_packed + node_off[g] + g;
        int32_t *ci = colidx_packed + cap_off[g];
        int64_t m;
        if (kind[g] == 1 && n > 0) {
            m = gg_rmat_csr(scale[g], n, param[g], 0.57, 0.19, 0.19, key[g], 1, rp, ci);
        } else if (kind[g] == 0 && n > 1 && param[g] > 0) {
            m = gg_er_csr(n, param[g], key[g], rp, ci);
        } else { /* no edges */
            memset(rp, 0, sizeof(int32_t) * (size_t)(n + 1));
            m = 0;
        }
        m_out[g] = m;
        if (m < 0 || m > cap_off[g + 1] - cap_off[g]) {
#pragma omp critical
            if (!fail) fail = -1 - g;
        }
    }
    return fail;
}

/* Close the gaps left by gg_batch: move graph g's entries from cap_off[g] to edge_off[g]
 * (edge_off[g] <= cap_off[g], graphs in increasing order so nothing is overwritten early). */
void gg_batch_compact(int64_t G, const int64_t *cap_off, const int64_t *edge_off, int32_t *colidx_packed) {
    for (int64_t g = 0; g < G; ++g) {
        const int64_t len = edge_off[g + 1] - edge_off[g];
        if (len > 0 && edge_off[g] != cap_off[g])
            memmove(colidx_packed + edge_off[g], colidx_packed + cap_off[g], sizeof(int32_t) * (size_t)len);
    }
}
