/* Oracle setup: conflict graph, greedy colouring, CSR pattern, expected stamp map.
 * Written for clarity, independently of the GPU library's setup code.
 *
 * Conflict graph (Methodology): one vertex per FET; an edge joins two FETs that
 * share at least one non-ground node (optionally also skipping the nodes flagged
 * in `excl`).  Greedy colouring (Introduction): visit the FETs in ascending index
 * and give each the smallest colour not used by an already coloured neighbour.
 */
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#include "oracle_internal.h"

static int conflict_node(int32_t n, const uint8_t *excl) { return n != 0 && !(excl && excl[n]); }

int or_unique_nodes(const int32_t term4[4], int32_t u[4], int a[4]) {
    int k = 0;
    for (int t = 0; t < 4; ++t) {
        a[t] = -1;
        if (term4[t] == 0) continue;
        for (int j = 0; j < k; ++j)
            if (u[j] == term4[t]) { a[t] = j; break; }
        if (a[t] < 0) { u[k] = term4[t]; a[t] = k; ++k; }
    }
    return k;
}

int64_t or_find_slot(const int32_t *row_ptr, const int32_t *col_idx, int32_t r, int32_t c) {
    int64_t lo = row_ptr[r], hi = (int64_t)row_ptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (col_idx[mid] == c) return mid;
        if (col_idx[mid] < c) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

int or_colour(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl,
              int32_t *colour, int32_t *n_colours, int64_t *n_edges) {
    /* incidence lists: conflict node -> devices on it, ascending, each device once */
    int64_t *cnt = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int32_t v = 0; v < n_dev; ++v) {
        int32_t u[4]; int a[4];
        int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
        for (int j = 0; j < k; ++j) {
            if (u[j] < 0 || u[j] >= n_nodes) { free(cnt); return -2; }
            if (conflict_node(u[j], excl)) cnt[u[j] + 1]++;
        }
    }
    for (int32_t n = 0; n < n_nodes; ++n) cnt[n + 1] += cnt[n];
    int32_t *inc = malloc(sizeof(int32_t) * (size_t)(cnt[n_nodes] + 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    int64_t *forbid = malloc(sizeof(int64_t) * ((size_t)n_dev + 1));
    int64_t *seen = malloc(sizeof(int64_t) * ((size_t)n_dev + 1));
    if (!inc || !fill || !forbid || !seen) { free(cnt); free(inc); free(fill); free(forbid); free(seen); return -1; }
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int32_t v = 0; v < n_dev; ++v) {
        int32_t u[4]; int a[4];
        int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
        for (int j = 0; j < k; ++j)
            if (conflict_node(u[j], excl)) inc[fill[u[j]]++] = v;
    }
    for (int32_t v = 0; v <= n_dev; ++v) { forbid[v] = -1; seen[v] = -1; }

    int64_t edges = 0;
    int32_t C = 0;
    for (int32_t v = 0; v < n_dev; ++v) {
        int32_t u[4]; int a[4];
        int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
        for (int j = 0; j < k; ++j) {
            if (!conflict_node(u[j], excl)) continue;
            for (int64_t e = cnt[u[j]]; e < cnt[u[j] + 1]; ++e) {
                int32_t w = inc[e];
                if (w >= v) break;                 /* lists are ascending */
                forbid[colour[w]] = v;
                if (seen[w] != v) { seen[w] = v; ++edges; }
            }
        }
        int32_t c = 0;
        while (forbid[c] == v) ++c;
        colour[v] = c;
        if (c + 1 > C) C = c + 1;
    }
    if (n_colours) *n_colours = C;
    if (n_edges) *n_edges = edges;
    free(cnt); free(inc); free(fill); free(forbid); free(seen);
    return 0;
}

static int cmp_i64(const void *x, const void *y) {
    int64_t a = *(const int64_t *)x, b = *(const int64_t *)y;
    return (a > b) - (a < b);
}

/* MNA pattern: non-ground node n -> row n-1; voltage-source branch j -> row
 * (n_nodes-1)+j.  Entries: every ordered pair of a device's non-ground terminal
 * nodes, every node-row diagonal, (pos,br), (br,pos) (and neg likewise when
 * non-ground) for each voltage source, and (p,q), (q,p) for each series resistor
 * between non-ground nodes p and q.  Columns ascending and unique. */
int or_pattern(int32_t n_nodes, int32_t n_dev, const int32_t *term, int32_t n_vsrc,
               const int32_t *vsrc, int32_t n_res, const int32_t *res, int32_t *row_ptr,
               int32_t *col_idx, int64_t *nnz) {
    const int64_t n_rows = (int64_t)n_nodes - 1 + n_vsrc;
    const int64_t cap = 16 * (int64_t)n_dev + n_rows + 4 * (int64_t)n_vsrc + 2 * (int64_t)n_res;
    int64_t *key = malloc(sizeof(int64_t) * (size_t)(cap + 1));
    if (!key) return -1;
    int64_t m = 0;
    for (int32_t v = 0; v < n_dev; ++v)
        for (int t = 0; t < 4; ++t)
            for (int s = 0; s < 4; ++s) {
                int32_t r = term[4 * (int64_t)v + t], c = term[4 * (int64_t)v + s];
                if (r == 0 || c == 0) continue;
                key[m++] = (int64_t)(r - 1) * n_rows + (c - 1);
            }
    for (int64_t r = 0; r < (int64_t)n_nodes - 1; ++r) key[m++] = r * n_rows + r;
    for (int32_t j = 0; j < n_vsrc; ++j) {
        int64_t br = (int64_t)n_nodes - 1 + j;
        for (int e = 0; e < 2; ++e) {
            int32_t nd = vsrc[2 * j + e];
            if (nd == 0) continue;
            key[m++] = (int64_t)(nd - 1) * n_rows + br;
            key[m++] = br * n_rows + (nd - 1);
        }
    }
    /* series resistors: the off-diagonal pair between their two nodes */
    for (int32_t j = 0; j < n_res; ++j) {
        int32_t p = res[2 * (int64_t)j], q = res[2 * (int64_t)j + 1];
        if (p == 0 || q == 0) continue;
        key[m++] = (int64_t)(p - 1) * n_rows + (q - 1);
        key[m++] = (int64_t)(q - 1) * n_rows + (p - 1);
    }
    qsort(key, (size_t)m, sizeof(int64_t), cmp_i64);
    int64_t w = 0;
    for (int64_t i = 0; i < m; ++i)
        if (i == 0 || key[i] != key[i - 1]) key[w++] = key[i];
    for (int64_t r = 0; r <= n_rows; ++r) row_ptr[r] = 0;
    for (int64_t i = 0; i < w; ++i) {
        row_ptr[key[i] / n_rows + 1]++;
        col_idx[i] = (int32_t)(key[i] % n_rows);
    }
    for (int64_t r = 0; r < n_rows; ++r) row_ptr[r + 1] += row_ptr[r];
    *nnz = w;
    free(key);
    return 0;
}

/* Expected stamp map.  For device v with k unique non-ground nodes u[0..k-1]
 * (first appearance over d, g, s, b): slot j = a*k + b is the CSR position of
 * (u[a]-1, u[b]-1); b-row a is u[a]-1.  Hub entries: both nodes excluded (A) or the
 * node excluded (b).  Every other entry is a store for the writer of smallest
 * colour and an add for the rest; two writers of a non-hub entry never share a
 * colour (they share that entry's non-excluded node) - checked here. */
int or_stamp_map(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl,
                 const int32_t *colour, const int32_t *row_ptr, const int32_t *col_idx,
                 int32_t *slot, int8_t *sflag, int32_t *brow, int8_t *bflag) {
    const int64_t nnz = row_ptr[n_nodes - 1];   /* device entries lie in node rows */
    int32_t *minc = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    int32_t *minr = malloc(sizeof(int32_t) * (size_t)n_nodes);
    if (!minc || !minr) { free(minc); free(minr); return -1; }
    for (int64_t i = 0; i < nnz; ++i) minc[i] = -1;
    for (int32_t i = 0; i < n_nodes; ++i) minr[i] = -1;
    for (int pass = 0; pass < 2; ++pass) {
        for (int32_t v = 0; v < n_dev; ++v) {
            int32_t u[4]; int a[4];
            int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
            for (int j = 0; j < 16; ++j) { slot[16 * (int64_t)v + j] = -1; sflag[16 * (int64_t)v + j] = -1; }
            for (int j = 0; j < 4; ++j) { brow[4 * (int64_t)v + j] = -1; bflag[4 * (int64_t)v + j] = -1; }
            for (int r = 0; r < k; ++r) {
                for (int c = 0; c < k; ++c) {
                    int64_t s = or_find_slot(row_ptr, col_idx, u[r] - 1, u[c] - 1);
                    if (s < 0) { free(minc); free(minr); return -3; }
                    int hub = excl && excl[u[r]] && excl[u[c]];
                    slot[16 * (int64_t)v + r * k + c] = (int32_t)s;
                    if (hub) { sflag[16 * (int64_t)v + r * k + c] = 2; continue; }
                    if (pass == 0) {
                        if (minc[s] < 0 || colour[v] < minc[s]) minc[s] = colour[v];
                    } else {
                        sflag[16 * (int64_t)v + r * k + c] = colour[v] == minc[s] ? 1 : 0;
                    }
                }
                int hubr = excl && excl[u[r]];
                brow[4 * (int64_t)v + r] = u[r] - 1;
                if (hubr) { bflag[4 * (int64_t)v + r] = 2; continue; }
                if (pass == 0) {
                    if (minr[u[r]] < 0 || colour[v] < minr[u[r]]) minr[u[r]] = colour[v];
                } else {
                    bflag[4 * (int64_t)v + r] = colour[v] == minr[u[r]] ? 1 : 0;
                }
            }
        }
    }
    /* validity: exactly one store per written non-hub entry */
    int32_t *stores = calloc((size_t)nnz + (size_t)n_nodes + 1, sizeof(int32_t));
    int rc = 0;
    if (!stores) rc = -1;
    for (int32_t v = 0; v < n_dev && rc == 0; ++v) {
        for (int j = 0; j < 16; ++j)
            if (sflag[16 * (int64_t)v + j] == 1) stores[slot[16 * (int64_t)v + j]]++;
        for (int j = 0; j < 4; ++j)
            if (bflag[4 * (int64_t)v + j] == 1) stores[nnz + brow[4 * (int64_t)v + j]]++;
    }
    for (int64_t i = 0; i < nnz + n_nodes && rc == 0; ++i)
        if (stores[i] > 1) rc = -4;   /* two same-colour writers: invalid colouring */
    free(stores); free(minc); free(minr);
    return rc;
}

/* ---- colouring in other vertex orders (test infrastructure) -------------------
 * Explicit conflict graph (adjacency lists, each neighbour once), then:
 *   order 1, largest first (Welsh and Powell): vertices by decreasing degree, ties
 *     by ascending index, each given the smallest colour not used by an already
 *     coloured neighbour;
 *   order 2, DSATUR (Brelaz): repeatedly the uncoloured vertex with the most
 *     distinct colours among its neighbours, ties by larger degree, then smaller
 *     index, given the smallest colour not used by its neighbours.
 * Plain and quadratic: meant for the small graphs of the tests. */
static int build_adjacency(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl,
                           int64_t **adj_ptr, int32_t **adj) {
    int64_t *cnt = calloc((size_t)n_nodes + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int32_t v = 0; v < n_dev; ++v) {
        int32_t u[4]; int a[4];
        int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
        for (int j = 0; j < k; ++j) {
            if (u[j] < 0 || u[j] >= n_nodes) { free(cnt); return -2; }
            if (conflict_node(u[j], excl)) cnt[u[j] + 1]++;
        }
    }
    for (int32_t n = 0; n < n_nodes; ++n) cnt[n + 1] += cnt[n];
    int32_t *inc = malloc(sizeof(int32_t) * (size_t)(cnt[n_nodes] + 1));
    int64_t *fill = malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    int32_t *mark = malloc(sizeof(int32_t) * ((size_t)n_dev + 1));
    int64_t *ptr = calloc((size_t)n_dev + 1, sizeof(int64_t));
    if (!inc || !fill || !mark || !ptr) { free(cnt); free(inc); free(fill); free(mark); free(ptr); return -1; }
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int32_t v = 0; v < n_dev; ++v) {
        int32_t u[4]; int a[4];
        int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
        for (int j = 0; j < k; ++j)
            if (conflict_node(u[j], excl)) inc[fill[u[j]]++] = v;
    }
    /* two passes over every device's incident nodes: count, then fill */
    int32_t *list = NULL;
    for (int pass = 0; pass < 2; ++pass) {
        for (int32_t v = 0; v <= n_dev; ++v) mark[v] = -1;
        for (int32_t v = 0; v < n_dev; ++v) {
            int32_t u[4]; int a[4];
            int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
            int64_t d = 0;
            for (int j = 0; j < k; ++j) {
                if (!conflict_node(u[j], excl)) continue;
                for (int64_t e = cnt[u[j]]; e < cnt[u[j] + 1]; ++e) {
                    int32_t w = inc[e];
                    if (w == v || mark[w] == v) continue;
                    mark[w] = v;
                    if (pass == 1) list[ptr[v] + d] = w;
                    ++d;
                }
            }
            if (pass == 0) ptr[v + 1] = d;
        }
        if (pass == 0) {
            for (int32_t v = 0; v < n_dev; ++v) ptr[v + 1] += ptr[v];
            list = malloc(sizeof(int32_t) * (size_t)(ptr[n_dev] + 1));
            if (!list) { free(cnt); free(inc); free(fill); free(mark); free(ptr); return -1; }
        }
    }
    free(cnt); free(inc); free(fill); free(mark);
    *adj_ptr = ptr;
    *adj = list;
    return 0;
}

/* smallest colour not used by a coloured neighbour of v (colour -1 = none yet) */
static int32_t smallest_free(const int64_t *ptr, const int32_t *adj, const int32_t *colour, int32_t v,
                             int32_t *stamp, int32_t tag) {
    for (int64_t e = ptr[v]; e < ptr[v + 1]; ++e)
        if (colour[adj[e]] >= 0) stamp[colour[adj[e]]] = tag;
    int32_t c = 0;
    while (stamp[c] == tag) ++c;
    return c;
}

int or_colour_order(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl, int order,
                    int32_t *colour, int32_t *n_colours, int64_t *n_edges) {
    if (order == 0) return or_colour(n_nodes, n_dev, term, excl, colour, n_colours, n_edges);
    if (order != 1 && order != 2) return -3;
    int64_t *ptr; int32_t *adj;
    int rc = build_adjacency(n_nodes, n_dev, term, excl, &ptr, &adj);
    if (rc) return rc;
    int32_t *stamp = malloc(sizeof(int32_t) * ((size_t)n_dev + 1));
    int32_t *sat = calloc((size_t)n_dev + 1, sizeof(int32_t));
    int32_t *seq = malloc(sizeof(int32_t) * ((size_t)n_dev + 1));
    if (!stamp || !sat || !seq) { free(ptr); free(adj); free(stamp); free(sat); free(seq); return -1; }
    for (int32_t v = 0; v <= n_dev; ++v) stamp[v] = -1;
    for (int32_t v = 0; v < n_dev; ++v) colour[v] = -1;
    int32_t C = 0;
    if (order == 1) {
        /* insertion sort by (degree descending, index ascending): stable and plain */
        for (int32_t i = 0; i < n_dev; ++i) {
            int32_t v = i, j = i;
            int64_t dv = ptr[v + 1] - ptr[v];
            while (j > 0 && ptr[seq[j - 1] + 1] - ptr[seq[j - 1]] < dv) { seq[j] = seq[j - 1]; --j; }
            seq[j] = v;
        }
        for (int32_t i = 0; i < n_dev; ++i) {
            int32_t v = seq[i];
            colour[v] = smallest_free(ptr, adj, colour, v, stamp, i);
            if (colour[v] + 1 > C) C = colour[v] + 1;
        }
    } else {
        for (int32_t step = 0; step < n_dev; ++step) {
            int32_t best = -1;
            for (int32_t v = 0; v < n_dev; ++v) {
                if (colour[v] >= 0) continue;
                if (best < 0 || sat[v] > sat[best] ||
                    (sat[v] == sat[best] && ptr[v + 1] - ptr[v] > ptr[best + 1] - ptr[best]))
                    best = v;
            }
            int32_t c = smallest_free(ptr, adj, colour, best, stamp, step);
            colour[best] = c;
            if (c + 1 > C) C = c + 1;
            /* saturation: a neighbour gains one when c is new among its coloured
             * neighbours (best is now one of them) */
            for (int64_t e = ptr[best]; e < ptr[best + 1]; ++e) {
                int32_t u = adj[e];
                if (colour[u] >= 0) continue;
                int seen = 0;
                for (int64_t f = ptr[u]; f < ptr[u + 1]; ++f)
                    if (adj[f] != best && colour[adj[f]] == c) { seen = 1; break; }
                if (!seen) sat[u]++;
            }
        }
    }
    if (n_colours) *n_colours = C;
    if (n_edges) *n_edges = ptr[n_dev] / 2;
    free(ptr); free(adj); free(stamp); free(sat); free(seq);
    return 0;
}
