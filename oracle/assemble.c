/* Oracle assembly of the MNA matrix values A (fixed CSR pattern) and RHS b.
 *
 * Stamp phase (Methodology): every device's contributions are accumulated into
 * the shared A and b.  Two accumulation orders are provided:
 *   serial  - devices ascending, A and b start at zero, each contribution added
 *             (the single-thread baseline of the kernel-variants table);
 *   replay  - colours ascending (Methodology: colours processed sequentially);
 *             within a colour no two devices share a non-hub entry, so the order
 *             inside a colour is irrelevant.  The first writer of an entry stores,
 *             later writers add.  Entries of excluded (hub) nodes are summed by the
 *             fixed-shape pairwise or_hubsum over the contributions in ascending
 *             device index.
 * Per device, the 4x4 local matrix Y is merged onto its unique node pairs: each
 * merged value is the left-to-right sum of the Y entries mapping to it in (t, u)
 * row-major order over (d, g, s, b); b rows likewise in terminal order.
 * The series resistors of a split netlist (Benchmark 2, Table I's R rows) are linear:
 * their stamps form a constant per-entry sum (or_linear_stamp) that is added once to
 * each entry they touch, after all device contributions, in both orders.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "oracle.h"
#include "oracle_internal.h"

/* HubSum: the pairwise (tree) sum of m contributions, split at the largest power of
 * two below m: HubSum(c, m) = HubSum(c, h) + HubSum(c + h, m - h), h = 2^ceil(log2 m) / 2,
 * and HubSum(c, 1) = c[0].  Equivalently a perfect binary tree over the contributions
 * padded with -0.0 to a power of two (x + -0.0 = x exactly).  Every aligned block of
 * 2^k contributions is a subtree of its own, so the sum can be formed block by block. */
double or_hubsum(const double *c, int64_t m) {
    if (m <= 0) return 0.0;
    if (m == 1) return c[0];
    int64_t h = 1;
    while (2 * h < m) h *= 2;
    return or_hubsum(c, h) + or_hubsum(c + h, m - h);
}

/* Merge a device's Y and bl onto its unique nodes. mA[a*k+b], mB[a]. */
static int merge_device(const int32_t term4[4], const double Y[16], const double bl[4],
                        double mA[16], double mB[4]) {
    int32_t u[4]; int a[4];
    int k = or_unique_nodes(term4, u, a);
    int initA[16] = {0}, initB[4] = {0};
    for (int t = 0; t < 4; ++t) {
        if (a[t] < 0) continue;
        for (int s = 0; s < 4; ++s) {
            if (a[s] < 0) continue;
            int j = a[t] * k + a[s];
            if (!initA[j]) { mA[j] = Y[t * 4 + s]; initA[j] = 1; }
            else mA[j] = mA[j] + Y[t * 4 + s];
        }
        if (!initB[a[t]]) { mB[a[t]] = bl[t]; initB[a[t]] = 1; }
        else mB[a[t]] = mB[a[t]] + bl[t];
    }
    return k;
}

static void gather_v(const int32_t term4[4], const double *x, double V[4]) {
    for (int t = 0; t < 4; ++t) V[t] = term4[t] == 0 ? 0.0 : x[term4[t] - 1];
}

typedef struct { int64_t key; int32_t dev; double val; } hub_item;

static int cmp_hub(const void *x, const void *y) {
    const hub_item *a = x, *b = y;
    if (a->key != b->key) return (a->key > b->key) - (a->key < b->key);
    return (a->dev > b->dev) - (a->dev < b->dev);
}

int or_linear_stamp(int32_t n_nodes, int32_t n_res, const int32_t *res, const double *g,
                    const int32_t *row_ptr, const int32_t *col_idx, int64_t nnz, double *Lin,
                    uint8_t *touched, int magnitude) {
    for (int64_t i = 0; i < nnz; ++i) { Lin[i] = 0.0; touched[i] = 0; }
    for (int32_t j = 0; j < n_res; ++j) {
        const int32_t nd[2] = {res[2 * (int64_t)j], res[2 * (int64_t)j + 1]};
        if (nd[0] < 0 || nd[0] >= n_nodes || nd[1] < 0 || nd[1] >= n_nodes) return -2;
        /* +g on the diagonals, -g between the two nodes, in (p,p) (p,q) (q,p) (q,q) order */
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 2; ++c) {
                if (nd[r] == 0 || nd[c] == 0) continue;
                int64_t s = or_find_slot(row_ptr, col_idx, nd[r] - 1, nd[c] - 1);
                if (s < 0) return -3;
                double v = r == c ? g[j] : -g[j];
                Lin[s] = Lin[s] + (magnitude ? fabs(v) : v);
                touched[s] = 1;
            }
    }
    return 0;
}

static int assemble_impl(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                         int32_t n_vsrc, const int32_t *vsrc, const double *vsrc_volts,
                         int32_t n_res, const int32_t *res, const double *res_g,
                         const or_card *nmos, const or_card *pmos, const double *W,
                         const double *L, const double *VTH0, const int32_t *row_ptr,
                         const int32_t *col_idx, const int32_t *colour, const uint8_t *excl,
                         const double *x, double ag0, const double *hist, double *A, double *b,
                         int magnitude) {
    const int64_t n_rows = (int64_t)n_nodes - 1 + n_vsrc;
    const int64_t nnz = row_ptr[n_rows];
    double *mA = malloc(sizeof(double) * 16 * ((size_t)n_dev + 1));
    double *mB = malloc(sizeof(double) * 4 * ((size_t)n_dev + 1));
    int64_t *sl = malloc(sizeof(int64_t) * 16 * ((size_t)n_dev + 1));
    int *kk = malloc(sizeof(int) * ((size_t)n_dev + 1));
    if (!mA || !mB || !sl || !kk) { free(mA); free(mB); free(sl); free(kk); return -1; }

    /* compute phase: every device, local values merged onto its node pairs */
    for (int32_t v = 0; v < n_dev; ++v) {
        const int32_t *t4 = term + 4 * (int64_t)v;
        double V[4], Y[16], bl[4], Icur[4], Q[4];
        gather_v(t4, x, V);
        or_device_eval(pol[v] > 0 ? nmos : pmos, pol[v], W[v], L[v], VTH0[v], V, ag0,
                       hist ? hist + 4 * (int64_t)v : NULL, Y, bl, Icur, Q, NULL);
        kk[v] = merge_device(t4, Y, bl, mA + 16 * (int64_t)v, mB + 4 * (int64_t)v);
        int32_t u[4]; int a[4];
        or_unique_nodes(t4, u, a);
        for (int r = 0; r < kk[v]; ++r)
            for (int c = 0; c < kk[v]; ++c) {
                int64_t s = or_find_slot(row_ptr, col_idx, u[r] - 1, u[c] - 1);
                if (s < 0) { free(mA); free(mB); free(sl); free(kk); return -3; }
                sl[16 * (int64_t)v + r * kk[v] + c] = s;
            }
    }

    for (int64_t i = 0; i < nnz; ++i) A[i] = 0.0;
    for (int64_t i = 0; i < n_rows; ++i) b[i] = 0.0;
    /* voltage sources: branch current into pos (out of neg); V(pos) - V(neg) = V */
    for (int32_t j = 0; j < n_vsrc; ++j) {
        int32_t br = n_nodes - 1 + j;
        for (int e = 0; e < 2; ++e) {
            int32_t nd = vsrc[2 * j + e];
            if (nd == 0) continue;
            double sgn = e == 0 ? 1.0 : -1.0;
            A[or_find_slot(row_ptr, col_idx, nd - 1, br)] = sgn;
            A[or_find_slot(row_ptr, col_idx, br, nd - 1)] = sgn;
        }
        b[br] = vsrc_volts[j];
    }

    if (!colour) {
        for (int32_t v = 0; v < n_dev; ++v) {
            int32_t u[4]; int a[4];
            or_unique_nodes(term + 4 * (int64_t)v, u, a);
            for (int j = 0; j < kk[v] * kk[v]; ++j) {
                double m = mA[16 * (int64_t)v + j];
                A[sl[16 * (int64_t)v + j]] += magnitude ? fabs(m) : m;
            }
            for (int r = 0; r < kk[v]; ++r) {
                double m = mB[4 * (int64_t)v + r];
                b[u[r] - 1] += magnitude ? fabs(m) : m;
            }
        }
    } else {
        int32_t C = 0;
        for (int32_t v = 0; v < n_dev; ++v) if (colour[v] + 1 > C) C = colour[v] + 1;
        char *doneA = calloc((size_t)nnz + 1, 1), *doneB = calloc((size_t)n_rows + 1, 1);
        hub_item *hubs = malloc(sizeof(hub_item) * (20 * (size_t)n_dev + 1));
        int64_t nh = 0;
        /* devices grouped by colour, ascending index inside a colour */
        int64_t *cptr = calloc((size_t)C + 1, sizeof(int64_t));
        int32_t *order = malloc(sizeof(int32_t) * ((size_t)n_dev + 1));
        for (int32_t v = 0; v < n_dev; ++v) cptr[colour[v] + 1]++;
        for (int32_t c = 0; c < C; ++c) cptr[c + 1] += cptr[c];
        int64_t *fillp = malloc(sizeof(int64_t) * ((size_t)C + 1));
        memcpy(fillp, cptr, sizeof(int64_t) * ((size_t)C + 1));
        for (int32_t v = 0; v < n_dev; ++v) order[fillp[colour[v]]++] = v;
        for (int32_t c = 0; c < C; ++c) {
            for (int64_t e = cptr[c]; e < cptr[c + 1]; ++e) {
                int32_t v = order[e];
                int32_t u[4]; int a[4];
                int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
                for (int r = 0; r < k; ++r) {
                    for (int cc = 0; cc < k; ++cc) {
                        int64_t s = sl[16 * (int64_t)v + r * k + cc];
                        double m = mA[16 * (int64_t)v + r * k + cc];
                        if (excl && excl[u[r]] && excl[u[cc]]) {
                            hubs[nh].key = s; hubs[nh].dev = v; hubs[nh].val = m; ++nh;
                        } else if (!doneA[s]) { A[s] = m; doneA[s] = 1; }
                        else A[s] = A[s] + m;
                    }
                    int64_t row = u[r] - 1;
                    double mb = mB[4 * (int64_t)v + r];
                    if (excl && excl[u[r]]) {
                        hubs[nh].key = nnz + row; hubs[nh].dev = v; hubs[nh].val = mb; ++nh;
                    } else if (!doneB[row]) { b[row] = mb; doneB[row] = 1; }
                    else b[row] = b[row] + mb;
                }
            }
        }
        /* hub outputs: contributions in ascending device index, fixed-shape sum */
        qsort(hubs, (size_t)nh, sizeof(hub_item), cmp_hub);
        double *vals = malloc(sizeof(double) * ((size_t)nh + 1));
        for (int64_t i = 0; i < nh;) {
            int64_t j = i;
            while (j < nh && hubs[j].key == hubs[i].key) { vals[j - i] = hubs[j].val; ++j; }
            double s = or_hubsum(vals, j - i);
            if (hubs[i].key < nnz) A[hubs[i].key] = s; else b[hubs[i].key - nnz] = s;
            i = j;
        }
        free(vals); free(doneA); free(doneB); free(hubs); free(cptr); free(order); free(fillp);
    }
    free(mA); free(mB); free(sl); free(kk);
    /* linear part, added once per entry after every device contribution */
    if (n_res > 0) {
        double *Lin = malloc(sizeof(double) * ((size_t)nnz + 1));
        uint8_t *touched = malloc((size_t)nnz + 1);
        if (!Lin || !touched) { free(Lin); free(touched); return -1; }
        int rc = or_linear_stamp(n_nodes, n_res, res, res_g, row_ptr, col_idx, nnz, Lin, touched,
                                 magnitude);
        if (rc == 0)
            for (int64_t i = 0; i < nnz; ++i)
                if (touched[i]) A[i] = A[i] + Lin[i];
        free(Lin); free(touched);
        return rc;
    }
    return 0;
}

int or_assemble(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                int32_t n_vsrc, const int32_t *vsrc, const double *vsrc_volts,
                int32_t n_res, const int32_t *res, const double *res_g, const or_card *nmos,
                const or_card *pmos, const double *W, const double *L, const double *VTH0,
                const int32_t *row_ptr, const int32_t *col_idx, const int32_t *colour,
                const uint8_t *excl, const double *x, double ag0, const double *hist, double *A,
                double *b) {
    return assemble_impl(n_nodes, n_dev, term, pol, n_vsrc, vsrc, vsrc_volts, n_res, res, res_g, nmos,
                         pmos, W, L, VTH0, row_ptr, col_idx, colour, excl, x, ag0, hist, A, b, 0);
}

/* Sum of |contribution| per entry (serial), the natural scale of a reordered sum. */
int or_assemble_magnitude(int32_t n_nodes, int32_t n_dev, const int32_t *term,
                          const int8_t *pol, int32_t n_vsrc, const int32_t *vsrc,
                          const double *vsrc_volts, int32_t n_res, const int32_t *res,
                          const double *res_g, const or_card *nmos, const or_card *pmos,
                          const double *W, const double *L, const double *VTH0,
                          const int32_t *row_ptr, const int32_t *col_idx, const double *x,
                          double ag0, const double *hist, double *A, double *b) {
    return assemble_impl(n_nodes, n_dev, term, pol, n_vsrc, vsrc, vsrc_volts, n_res, res, res_g, nmos,
                         pmos, W, L, VTH0, row_ptr, col_idx, NULL, NULL, x, ag0, hist, A, b, 1);
}

/* Colour replay on every host core (the paper's ColorFused on its CPU: per-colour
 * parallel for over the devices of the colour).  Same values as the serial colour
 * replay, bit for bit: the compute phase is per device; within a colour no two
 * devices share a non-hub entry, so each entry still receives its contributions in
 * colour order (first writer stores, later writers add); hub contributions go to
 * per-device places and are summed by or_hubsum in ascending device index, as in
 * the serial replay.  Threads: the OpenMP default (OMP_NUM_THREADS). */
int or_assemble_omp(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                    int32_t n_vsrc, const int32_t *vsrc, const double *vsrc_volts,
                    int32_t n_res, const int32_t *res, const double *res_g, const or_card *nmos,
                    const or_card *pmos, const double *W, const double *L, const double *VTH0,
                    const int32_t *row_ptr, const int32_t *col_idx, const int32_t *colour,
                    const uint8_t *excl, const double *x, double ag0, const double *hist, double *A,
                    double *b) {
    const int64_t n_rows = (int64_t)n_nodes - 1 + n_vsrc;
    const int64_t nnz = row_ptr[n_rows];
    double *mA = malloc(sizeof(double) * 16 * ((size_t)n_dev + 1));
    double *mB = malloc(sizeof(double) * 4 * ((size_t)n_dev + 1));
    int64_t *sl = malloc(sizeof(int64_t) * 16 * ((size_t)n_dev + 1));
    int *kk = malloc(sizeof(int) * ((size_t)n_dev + 1));
    int64_t *hoff = malloc(sizeof(int64_t) * ((size_t)n_dev + 1));
    int bad = 0;
    if (!mA || !mB || !sl || !kk || !hoff) { free(mA); free(mB); free(sl); free(kk); free(hoff); return -1; }
    /* the operation counter counts serial evaluations only */
    const int counting = or_counting_;
    or_counting_ = 0;

    /* compute phase, one device per iteration */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int32_t v = 0; v < n_dev; ++v) {
        const int32_t *t4 = term + 4 * (int64_t)v;
        double V[4], Y[16], bl[4], Icur[4], Q[4];
        gather_v(t4, x, V);
        or_device_eval(pol[v] > 0 ? nmos : pmos, pol[v], W[v], L[v], VTH0[v], V, ag0,
                       hist ? hist + 4 * (int64_t)v : NULL, Y, bl, Icur, Q, NULL);
        kk[v] = merge_device(t4, Y, bl, mA + 16 * (int64_t)v, mB + 4 * (int64_t)v);
        int32_t u[4]; int a[4];
        or_unique_nodes(t4, u, a);
        for (int r = 0; r < kk[v]; ++r)
            for (int c = 0; c < kk[v]; ++c) {
                int64_t s = or_find_slot(row_ptr, col_idx, u[r] - 1, u[c] - 1);
                if (s < 0) bad = 1;
                sl[16 * (int64_t)v + r * kk[v] + c] = s;
            }
    }
    or_counting_ = counting;
    if (bad) { free(mA); free(mB); free(sl); free(kk); free(hoff); return -3; }

    for (int64_t i = 0; i < nnz; ++i) A[i] = 0.0;
    for (int64_t i = 0; i < n_rows; ++i) b[i] = 0.0;
    for (int32_t j = 0; j < n_vsrc; ++j) {
        int32_t br = n_nodes - 1 + j;
        for (int e = 0; e < 2; ++e) {
            int32_t nd = vsrc[2 * j + e];
            if (nd == 0) continue;
            double sgn = e == 0 ? 1.0 : -1.0;
            A[or_find_slot(row_ptr, col_idx, nd - 1, br)] = sgn;
            A[or_find_slot(row_ptr, col_idx, br, nd - 1)] = sgn;
        }
        b[br] = vsrc_volts[j];
    }

    /* hub places per device: prefix over the devices in ascending index */
    int64_t nh = 0;
    for (int32_t v = 0; v < n_dev; ++v) {
        hoff[v] = nh;
        int32_t u[4]; int a[4];
        int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
        for (int r = 0; r < k; ++r) {
            if (!(excl && excl[u[r]])) continue;
            for (int c = 0; c < k; ++c) nh += excl[u[c]] ? 1 : 0;
            nh += 1;
        }
    }
    int32_t C = 0;
    for (int32_t v = 0; v < n_dev; ++v) if (colour[v] + 1 > C) C = colour[v] + 1;
    char *doneA = calloc((size_t)nnz + 1, 1), *doneB = calloc((size_t)n_rows + 1, 1);
    hub_item *hubs = malloc(sizeof(hub_item) * ((size_t)nh + 1));
    int64_t *cptr = calloc((size_t)C + 1, sizeof(int64_t));
    int32_t *order = malloc(sizeof(int32_t) * ((size_t)n_dev + 1));
    int64_t *fillp = malloc(sizeof(int64_t) * ((size_t)C + 1));
    for (int32_t v = 0; v < n_dev; ++v) cptr[colour[v] + 1]++;
    for (int32_t c = 0; c < C; ++c) cptr[c + 1] += cptr[c];
    memcpy(fillp, cptr, sizeof(int64_t) * ((size_t)C + 1));
    for (int32_t v = 0; v < n_dev; ++v) order[fillp[colour[v]]++] = v;
    for (int32_t c = 0; c < C; ++c) {
        /* the devices of one colour touch disjoint non-hub entries */
#pragma omp parallel for schedule(static)
        for (int64_t e = cptr[c]; e < cptr[c + 1]; ++e) {
            int32_t v = order[e];
            int32_t u[4]; int a[4];
            int k = or_unique_nodes(term + 4 * (int64_t)v, u, a);
            int64_t h = hoff[v];
            for (int r = 0; r < k; ++r) {
                for (int cc = 0; cc < k; ++cc) {
                    int64_t s = sl[16 * (int64_t)v + r * k + cc];
                    double m = mA[16 * (int64_t)v + r * k + cc];
                    if (excl && excl[u[r]] && excl[u[cc]]) {
                        hubs[h].key = s; hubs[h].dev = v; hubs[h].val = m; ++h;
                    } else if (!doneA[s]) { A[s] = m; doneA[s] = 1; }
                    else A[s] = A[s] + m;
                }
                int64_t row = u[r] - 1;
                double mb = mB[4 * (int64_t)v + r];
                if (excl && excl[u[r]]) {
                    hubs[h].key = nnz + row; hubs[h].dev = v; hubs[h].val = mb; ++h;
                } else if (!doneB[row]) { b[row] = mb; doneB[row] = 1; }
                else b[row] = b[row] + mb;
            }
        }
    }
    qsort(hubs, (size_t)nh, sizeof(hub_item), cmp_hub);
    double *vals = malloc(sizeof(double) * ((size_t)nh + 1));
    for (int64_t i = 0; i < nh;) {
        int64_t j = i;
        while (j < nh && hubs[j].key == hubs[i].key) { vals[j - i] = hubs[j].val; ++j; }
        double s = or_hubsum(vals, j - i);
        if (hubs[i].key < nnz) A[hubs[i].key] = s; else b[hubs[i].key - nnz] = s;
        i = j;
    }
    free(vals); free(doneA); free(doneB); free(hubs); free(cptr); free(order); free(fillp);
    free(mA); free(mB); free(sl); free(kk); free(hoff);
    if (n_res > 0) {
        double *Lin = malloc(sizeof(double) * ((size_t)nnz + 1));
        uint8_t *touched = malloc((size_t)nnz + 1);
        if (!Lin || !touched) { free(Lin); free(touched); return -1; }
        int rc = or_linear_stamp(n_nodes, n_res, res, res_g, row_ptr, col_idx, nnz, Lin, touched, 0);
        if (rc == 0)
            for (int64_t i = 0; i < nnz; ++i)
                if (touched[i]) A[i] = A[i] + Lin[i];
        free(Lin); free(touched);
        return rc;
    }
    return 0;
}

int or_omp_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
