// Sparse LU refactorisation and triangular solves of the Newton loop, scheduled by
// dependency levels of the factor pattern (host analysis in newton.cpp).
//
// T holds (L - I) + U of P A Q in CSR over the permuted indices (columns ascending,
// pattern closed under fill).  Row i of L depends on the rows j < i with L(i, j) != 0;
// the rows of one lower level depend only on earlier levels, so each level is one
// launch with one lane per row.  A lane eliminates its row left to right: for each
// L entry (column j, ascending) it divides by U(j, j) and subtracts l * U(j, k) from
// its own entries k > j (a merge of two sorted column lists), and it carries the
// forward substitution y_i = b_P(i) - sum_j L(i, j) y_j along.  Rows up to
// LU_STAGE entries go to k_lu_lower_wave instead: one wave per row, the row staged
// in LDS, the lanes splitting U(j, :) and finding their columns in the row by
// binary search; every entry still receives its updates in ascending j, so both
// kernels give the same bits.  Rows within the caps of k_lu_lower_seq (most rows of
// circuit matrices) go to it instead: per row a wave first stages everything the
// row's elimination reads (the pivots, y_j and the U entries of its L rows that meet
// the row, their positions in the row found by the host), in one round of
// independent loads, so the sequential part runs from LDS; same operations in the
// same order.  A level launches one such wave per row; a run of consecutive narrow
// levels (a dependency chain, typical of the last rows of a minimum-degree order) is
// one launch of one wave that takes the run's rows one after another.  The backward
// substitution runs over upper levels, one workgroup per row (a rail's row of U can
// span the whole matrix), z_i = (y_i - sum_k U(i, k) z_k) / U(i, i), written to the
// solution at column Q(i).  Every sum has a fixed order for a fixed launch shape.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "launch.hpp"

namespace cs {

namespace {

constexpr int UPPER_BLOCK = 256;
constexpr int32_t LU_STAGE = 2048;   // row entries a wave stages in LDS (24 KiB)
constexpr int32_t SEQ_ROW = 256, SEQ_L = 64, SEQ_U = 256;   // k_lu_lower_seq caps per row

__global__ void __launch_bounds__(256) k_lu_load(int32_t nnzT, const int32_t *__restrict__ src,
                                                 const double *__restrict__ A, double *__restrict__ T) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nnzT) {
        const int32_t e = src[t];
        T[t] = e >= 0 ? A[e] : 0.0;
    }
}

__global__ void __launch_bounds__(256) k_lu_lower(int32_t count, const int32_t *__restrict__ rows,
                                                  const int32_t *__restrict__ Tp, const int32_t *__restrict__ Ti,
                                                  const int32_t *__restrict__ diag, double *T,
                                                  const int32_t *__restrict__ P, const double *__restrict__ b,
                                                  double *y) {
    const int32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= count) return;
    const int32_t i = rows[idx];
    const int32_t re = Tp[i + 1];
    double yi = b[P[i]];
    for (int32_t p = Tp[i]; p < diag[i]; ++p) {
        const int32_t j = Ti[p];
        const double l = T[p] / T[diag[j]];
        T[p] = l;
        yi = yi - l * y[j];
        int32_t q = diag[j] + 1, r = p + 1;
        const int32_t qe = Tp[j + 1];
        while (q < qe && r < re) {
            const int32_t kq = Ti[q], kr = Ti[r];
            if (kq == kr) {
                T[r] = T[r] - l * T[q];
                ++q;
                ++r;
            } else if (kq < kr) {
                ++q;
            } else {
                ++r;
            }
        }
    }
    y[i] = yi;
}

__global__ void __launch_bounds__(64) k_lu_lower_wave(const int32_t *__restrict__ rows,
                                                      const int32_t *__restrict__ Tp,
                                                      const int32_t *__restrict__ Ti,
                                                      const int32_t *__restrict__ diag, double *T,
                                                      const int32_t *__restrict__ P,
                                                      const double *__restrict__ b, double *y) {
    __shared__ double v[LU_STAGE];
    __shared__ int32_t col[LU_STAGE];
    const int32_t i = rows[blockIdx.x];
    const int32_t lane = threadIdx.x;
    const int32_t t0 = Tp[i], len = Tp[i + 1] - t0, nl = diag[i] - t0;
    for (int32_t r = lane; r < len; r += 64) {
        v[r] = T[t0 + r];
        col[r] = Ti[t0 + r];
    }
    __syncthreads();
    double yi = b[P[i]];
    // rows j of the L entries are final (earlier levels): the pivot, y_j, the end of
    // row j and this lane's first entry of U(j, :) are loaded one entry ahead
    struct Ahead {
        int32_t q0, qe, k0;
        double ujj, yj, t0;
    };
    auto fetch = [&](int32_t a) {
        Ahead f;
        const int32_t j = col[a];
        const int32_t dj = diag[j];
        f.q0 = dj + 1 + lane;
        f.qe = Tp[j + 1];
        f.ujj = T[dj];
        f.yj = y[j];
        f.k0 = f.q0 < f.qe ? Ti[f.q0] : -1;
        f.t0 = f.q0 < f.qe ? T[f.q0] : 0.0;
        return f;
    };
    Ahead cur{};
    if (nl > 0) cur = fetch(0);
    for (int32_t a = 0; a < nl; ++a) {
        const Ahead nxt = a + 1 < nl ? fetch(a + 1) : cur;
        const double l = v[a] / cur.ujj;
        yi = yi - l * cur.yj;
        __syncthreads();   // every lane has read v[a] before lane 0 replaces it
        if (lane == 0) v[a] = l;
        for (int32_t q = cur.q0; q < cur.qe; q += 64) {
            const int32_t k = q == cur.q0 ? cur.k0 : Ti[q];
            const double t = q == cur.q0 ? cur.t0 : T[q];
            int32_t lo = a + 1, hi = len;   // columns of the row after j, ascending
            while (lo < hi) {
                const int32_t m = (lo + hi) >> 1;
                if (col[m] < k) lo = m + 1;
                else hi = m;
            }
            if (lo < len && col[lo] == k) v[lo] = v[lo] - l * t;
        }
        __syncthreads();
        cur = nxt;
    }
    for (int32_t r = lane; r < len; r += 64) T[t0 + r] = v[r];
    if (lane == 0) y[i] = yi;
}

// Workgroup b (one wave) takes rows [b count, (b + 1) count) of the program in order,
// or rows [woff[b], woff[b + 1]) (each row's L columns are earlier rows of its own
// list or rows of earlier launches: a level is one workgroup per row, a run of narrow
// levels one workgroup per connected part of the L pattern), from a static program
// made by the host:
// prow (8 per row: row, T offset, entries, L entries, first L record, first staged
// record, staged records, b row P(i)), plo (3 per L entry: diagonal position of U(j, :),
// j, end of its staged records) and pst (2 per staged record: T position of U(j, k),
// position of column k in the row; only the k present in the row).  The program of
// the next row is loaded while the present one is eliminated; the values of a row
// (its entries, pivots, y_j, staged U entries) are one round of independent loads.
// Caps: SEQ_ROW entries, SEQ_L L entries, SEQ_U staged records per row.
struct SeqRow {
    int32_t i, t0, len, nl, lb, eb, ne, pi;
    int32_t dj, j, eend;
    int32_t q[SEQ_U / 64], pos[SEQ_U / 64];
};

__device__ inline SeqRow seq_fetch(const int32_t *__restrict__ prow, const int32_t *__restrict__ plo,
                                   const int32_t *__restrict__ pst, int32_t r, int32_t lane) {
    SeqRow f;
    const int32_t *h = prow + 8 * (size_t)r;
    f.i = h[0];
    f.t0 = h[1];
    f.len = h[2];
    f.nl = h[3];
    f.lb = h[4];
    f.eb = h[5];
    f.ne = h[6];
    f.pi = h[7];
    f.dj = f.j = f.eend = 0;
    if (lane < f.nl) {
        const int32_t *l = plo + 3 * (size_t)(f.lb + lane);
        f.dj = l[0];
        f.j = l[1];
        f.eend = l[2];
    }
#pragma unroll
    for (int u = 0; u < SEQ_U / 64; ++u) {
        const int32_t e = u * 64 + lane;
        f.q[u] = 0;
        f.pos[u] = 0;
        if (e < f.ne) {
            f.q[u] = pst[2 * (size_t)(f.eb + e)];
            f.pos[u] = pst[2 * (size_t)(f.eb + e) + 1];
        }
    }
    return f;
}

__global__ void __launch_bounds__(64) k_lu_lower_seq(int32_t count, const int32_t *__restrict__ woff,
                                                     const int32_t *__restrict__ prow,
                                                     const int32_t *__restrict__ plo,
                                                     const int32_t *__restrict__ pst, double *T,
                                                     const double *__restrict__ b, double *y) {
    __shared__ double v[SEQ_ROW];
    __shared__ double ut[SEQ_U];
    __shared__ int32_t upos[SEQ_U];
    __shared__ int32_t ubeg[SEQ_L + 1];
    __shared__ double ujj[SEQ_L], uy[SEQ_L];
    const int32_t lane = threadIdx.x;
    // workgroup b: rows [woff[b], woff[b + 1]) when woff is given, else [b count, (b + 1) count)
    const int32_t r_beg = woff ? woff[blockIdx.x] : (int32_t)blockIdx.x * count;
    count = woff ? woff[blockIdx.x + 1] - r_beg : count;
    if (count <= 0) return;
    prow += 8 * (size_t)r_beg;
    SeqRow cur = seq_fetch(prow, plo, pst, 0, lane);
    for (int32_t r = 0; r < count; ++r) {
        // values of this row: final except its own entries, which only it changes
        double vr[SEQ_ROW / 64], tq[SEQ_U / 64];
#pragma unroll
        for (int u = 0; u < SEQ_ROW / 64; ++u) {
            const int32_t e = u * 64 + lane;
            vr[u] = e < cur.len ? T[cur.t0 + e] : 0.0;
        }
        const double pj = lane < cur.nl ? T[cur.dj] : 1.0;
        const double yj = lane < cur.nl ? y[cur.j] : 0.0;
#pragma unroll
        for (int u = 0; u < SEQ_U / 64; ++u) tq[u] = u * 64 + lane < cur.ne ? T[cur.q[u]] : 0.0;
        double yi = b[cur.pi];
        const SeqRow nxt = r + 1 < count ? seq_fetch(prow, plo, pst, r + 1, lane) : cur;
#pragma unroll
        for (int u = 0; u < SEQ_ROW / 64; ++u)
            if (u * 64 + lane < cur.len) v[u * 64 + lane] = vr[u];
#pragma unroll
        for (int u = 0; u < SEQ_U / 64; ++u)
            if (u * 64 + lane < cur.ne) {
                ut[u * 64 + lane] = tq[u];
                upos[u * 64 + lane] = cur.pos[u];
            }
        if (lane < cur.nl) {
            ujj[lane] = pj;
            uy[lane] = yj;
            ubeg[lane + 1] = cur.eend;
        }
        if (lane == 0) ubeg[0] = 0;
        __syncthreads();
        for (int32_t a = 0; a < cur.nl; ++a) {
            const double l = v[a] / ujj[a];
            yi = yi - l * uy[a];
            __syncthreads();   // every lane has read v[a] before lane 0 replaces it
            if (lane == 0) v[a] = l;
            for (int32_t e = ubeg[a] + lane; e < ubeg[a + 1]; e += 64) {
                const int32_t pz = upos[e];
                v[pz] = v[pz] - l * ut[e];
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < SEQ_ROW / 64; ++u)
            if (u * 64 + lane < cur.len) T[cur.t0 + u * 64 + lane] = v[u * 64 + lane];
        if (lane == 0) y[cur.i] = yi;
        __syncthreads();   // this row's T and y are visible to the next rows of the run
        cur = nxt;
    }
}

__global__ void __launch_bounds__(UPPER_BLOCK) k_lu_upper(const int32_t *__restrict__ rows,
                                                          const int32_t *__restrict__ Tp,
                                                          const int32_t *__restrict__ Ti,
                                                          const int32_t *__restrict__ diag,
                                                          const double *__restrict__ T, double *y,
                                                          const int32_t *__restrict__ Q, double *out) {
    __shared__ double red[UPPER_BLOCK];
    const int32_t i = rows[blockIdx.x];
    double s = 0.0;
    for (int32_t p = diag[i] + 1 + (int32_t)threadIdx.x; p < Tp[i + 1]; p += UPPER_BLOCK) s = s + T[p] * y[Ti[p]];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = UPPER_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double z = (y[i] - red[0]) / T[diag[i]];
        y[i] = z;
        out[Q[i]] = z;
    }
}

// A run of consecutive upper levels in one workgroup of UPS_WAVES waves: per level,
// wave w takes the level's rows w, w + UPS_WAVES, ..., then a workgroup barrier makes
// the new z values visible to the next level.  Every row has at most UPPER_BLOCK
// entries right of the diagonal, and a wave forms its sum exactly as k_lu_upper's
// UPPER_BLOCK threads do (lane l holds the partial sums of threads l, l + 64, l + 128,
// l + 192 and the tree adds the same pairs in the same order): same bits.
constexpr int UPS_WAVES = 16;
__global__ void __launch_bounds__(64 * UPS_WAVES) k_lu_upper_seq(int32_t nlev, const int32_t *__restrict__ lev,
                                                                 const int32_t *__restrict__ rows,
                                                                 const int32_t *__restrict__ Tp,
                                                                 const int32_t *__restrict__ Ti,
                                                                 const int32_t *__restrict__ diag,
                                                                 const double *__restrict__ T, double *y,
                                                                 const int32_t *__restrict__ Q, double *out) {
    static_assert(UPPER_BLOCK == 256, "the tree below mirrors a 256-thread k_lu_upper");
    const int32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int32_t lv = 0; lv < nlev; ++lv) {
        const int32_t r1 = lev[lv + 1];
        for (int32_t k = lev[lv] + wave; k < r1; k += UPS_WAVES) {
            const int32_t i = rows[k];
            const int32_t d = diag[i], pe = Tp[i + 1];
            double s[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int32_t p = d + 1 + lane + 64 * m;   // thread lane + 64 m of k_lu_upper
                s[m] = 0.0;
                if (p < pe) s[m] = s[m] + T[p] * y[Ti[p]];
            }
            s[0] = s[0] + s[2];   // width 128
            s[1] = s[1] + s[3];
            double t = s[0] + s[1];   // width 64
            for (int w = 32; w > 0; w >>= 1) {
                const double o = __shfl_down(t, w, 64);
                if (lane < w) t = t + o;
            }
            if (lane == 0) {
                const double z = (y[i] - t) / T[d];
                y[i] = z;
                out[Q[i]] = z;
            }
        }
        __syncthreads();   // this level's z values are visible to the next level
    }
}

}  // namespace

hipError_t launch_lu_upper_seq(int32_t nlev, const int32_t *lev, const int32_t *rows, const int32_t *Tp,
                               const int32_t *Ti, const int32_t *diag, const double *T, double *y, const int32_t *Q,
                               double *out, hipStream_t s) {
    if (nlev <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_upper_seq, dim3(1), dim3(64 * UPS_WAVES), 0, s, nlev, lev, rows, Tp, Ti, diag, T, y, Q,
                       out);
    return hipGetLastError();
}

int32_t lu_upper_seq_rows() { return 4 * UPS_WAVES; }

hipError_t launch_lu_load(int32_t nnzT, const int32_t *src, const double *A, double *T, hipStream_t s) {
    if (nnzT <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_load, dim3((nnzT + 255) / 256), dim3(256), 0, s, nnzT, src, A, T);
    return hipGetLastError();
}

hipError_t launch_lu_lower(int32_t count, const int32_t *rows, const int32_t *Tp, const int32_t *Ti,
                           const int32_t *diag, double *T, const int32_t *P, const double *b, double *y,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_lower, dim3((count + 255) / 256), dim3(256), 0, s, count, rows, Tp, Ti, diag, T, P, b,
                       y);
    return hipGetLastError();
}

hipError_t launch_lu_lower_wave(int32_t count, const int32_t *rows, const int32_t *Tp, const int32_t *Ti,
                                const int32_t *diag, double *T, const int32_t *P, const double *b, double *y,
                                hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_lower_wave, dim3(count), dim3(64), 0, s, rows, Tp, Ti, diag, T, P, b, y);
    return hipGetLastError();
}

int32_t lu_stage_entries() { return LU_STAGE; }

void lu_seq_caps(int32_t *row, int32_t *l, int32_t *u) {
    *row = SEQ_ROW;
    *l = SEQ_L;
    *u = SEQ_U;
}

hipError_t launch_lu_lower_seq(int32_t grid, int32_t count, const int32_t *woff, const int32_t *prow,
                               const int32_t *plo, const int32_t *pst, double *T, const double *b, double *y,
                               hipStream_t s) {
    if (grid <= 0 || (!woff && count <= 0)) return hipSuccess;
    hipLaunchKernelGGL(k_lu_lower_seq, dim3(grid), dim3(64), 0, s, count, woff, prow, plo, pst, T, b, y);
    return hipGetLastError();
}

hipError_t launch_lu_upper(int32_t count, const int32_t *rows, const int32_t *Tp, const int32_t *Ti,
                           const int32_t *diag, const double *T, double *y, const int32_t *Q, double *out,
                           hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_lu_upper, dim3(count), dim3(UPPER_BLOCK), 0, s, rows, Tp, Ti, diag, T, y, Q, out);
    return hipGetLastError();
}

}  // namespace cs
