// Newton-Raphson loop around the evaluate-and-stamp path: the iteration the paper's
// method serves (Introduction: evaluate the devices at the present point, stamp the
// linearised MNA system, solve it for the next point), with the solve that the paper
// leaves to KLU (Benchmark 2; its Conclusions name the solver as the next
// bottleneck).
//
// Per iteration, on one stream: cs_eval_stamp (any variant), a sparse LU
// refactorisation of A with the pivots of one host factorisation (sparse_lu.cpp)
// and its two triangular solves (b becomes the Newton point y), then
// k_newton_update: d = y - x, node rows clamped to [-vstep, vstep], x += d, and the
// largest |d| read back to decide convergence (max |d| <= tol).  The refactorisation
// is either this library's level-scheduled kernels (solve.hip; levels, the rows'
// static elimination programs and the runs of narrow levels planned here once) or
// rocSOLVER's csrrf routines with the same pivots.  cs_batch_newton runs the same
// loop on a batch's block-diagonal system (every circuit of a sizing batch steps at
// once), with the node rows to clamp given by a per-row mask.
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "colorstamp.h"
#include "internal.hpp"
#include "launch.hpp"

namespace cs {

struct NewtonState {
    int device = -1;   // HIP device of the buffers below
    int32_t n = 0;
    int64_t nnzA = 0, nnzT = 0;
    DevBuf<int32_t> ptrA, indA, ptrT, indT, P, Q;
    DevBuf<double> valT;
    DevBuf<unsigned long long> step;
    DevBuf<uint8_t> clamp;   // rows whose step is clamped (batches; empty: rows below n_clamp)
    // level-scheduled refactorisation: T position -> A position (-1: fill), diagonal
    // positions, rows grouped by lower and by upper dependency level
    DevBuf<int32_t> src, diag, lrows, urows;
    DevBuf<double> y;
    // per lower level: programmed rows (listed first), then staged rows, then the rest
    std::vector<int32_t> lptr, uptr, lfit, lshort;
    // lower levels in launch order: [l0, l1) one level (l1 = l0 + 1) by the per-level
    // launches, or a run of narrow levels taken row after row by one k_lu_lower_seq wave
    struct LStep {
        int32_t l0, l1;
        bool seq;
        int32_t r0;        // first row of the step in the program
        int32_t w0 = 0;    // runs: first of grid + 1 workgroup row offsets in sq_woff
        int32_t grid = 1;  // runs: one workgroup per connected part of the L pattern
    };
    std::vector<LStep> lsteps;
    DevBuf<int32_t> sq_row, sq_lo, sq_st;   // the sequential program (k_lu_lower_seq)
    DevBuf<int32_t> sq_woff;                // runs: rows of each workgroup, relative to r0
    std::vector<LStep> usteps;   // upper levels: one launch per level, or a run in one workgroup
    DevBuf<int32_t> uptr_d;      // uptr on the device (level offsets of the upper runs)
    rocblas_handle handle = nullptr;   // rocSOLVER path, set up on its first use
    rocsolver_rfinfo rf = nullptr;
    double host_lu_ms = 0.0;
    ~NewtonState() {
        if (rf) (void)rocsolver_destroy_rfinfo(rf);
        if (handle) (void)rocblas_destroy_handle(handle);
    }
};

void destroy_newton(NewtonState *s) { delete s; }

}  // namespace cs

using namespace cs;

namespace {

cs_status nfail(cs_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

#define NCHECK_HIP(expr, what)                                                              \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return nfail(CS_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define NCHECK_RS(expr, what)                                                                   \
    do {                                                                                        \
        rocblas_status r_ = (expr);                                                             \
        if (r_ != rocblas_status_success)                                                       \
            return nfail(CS_EHIP, std::string(what) + ": rocSOLVER/rocBLAS status " + std::to_string((int)r_)); \
    } while (0)

struct Events {
    hipEvent_t e[5] = {};
    bool on = false;
    ~Events() {
        for (auto &v : e)
            if (v) (void)hipEventDestroy(v);
    }
};

// Host factorisation of the pattern m at the values of A (device), upload of the
// factor pattern and the level analysis and launch plan.  clamp (optional, host, m.n
// flags): rows whose Newton step is clamped.  flags: CS_NEWTON_NO_* bits.
cs_status build_state(const MnaView &m, int device, double *A_val, const std::vector<uint8_t> *clamp,
                      int32_t flags, hipStream_t s, NewtonState **out) {
    const int32_t n = m.n;
    const int64_t nnz = m.row_ptr[n];
    std::vector<double> Ah((size_t)nnz);
    NCHECK_HIP(hipMemcpyAsync(Ah.data(), A_val, sizeof(double) * Ah.size(), hipMemcpyDeviceToHost, s), "read A");
    NCHECK_HIP(hipStreamSynchronize(s), "stream synchronise");
    auto t0 = std::chrono::steady_clock::now();
    HostLU F;
    try {
        Err e = factor_mna(m, Ah.data(), F, nullptr);
        if (e.st != CS_OK) return nfail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return nfail(CS_ENOMEM, "host allocation");
    }
    auto ns = new (std::nothrow) NewtonState();
    if (!ns) return nfail(CS_ENOMEM, "host allocation");
    ns->host_lu_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ns->n = n;
    ns->device = device;
    ns->nnzA = nnz;
    ns->nnzT = (int64_t)F.Ti.size();
    struct Guard {
        NewtonState *p;
        ~Guard() { delete p; }
    } guard{ns};
    NCHECK_HIP(ns->ptrA.upload(std::vector<int32_t>(m.row_ptr, m.row_ptr + n + 1)), "upload pattern");
    NCHECK_HIP(ns->indA.upload(std::vector<int32_t>(m.col_idx, m.col_idx + nnz)), "upload pattern");
    NCHECK_HIP(ns->ptrT.upload(F.Tp), "upload factor pattern");
    NCHECK_HIP(ns->indT.upload(F.Ti), "upload factor pattern");
    NCHECK_HIP(ns->valT.upload(F.Tx), "upload factors");
    NCHECK_HIP(ns->P.upload(F.P), "upload pivots");
    NCHECK_HIP(ns->Q.upload(F.Q), "upload pivots");
    NCHECK_HIP(ns->step.alloc(1), "alloc step word");
    if (clamp) NCHECK_HIP(ns->clamp.upload(*clamp), "upload clamp flags");
    // level analysis of the factor pattern
    std::vector<int32_t> pinv((size_t)n), qinv((size_t)n), src((size_t)ns->nnzT, -1), diag((size_t)n, -1);
    for (int32_t k = 0; k < n; ++k) {
        pinv[(size_t)F.P[(size_t)k]] = k;
        qinv[(size_t)F.Q[(size_t)k]] = k;
    }
    for (int32_t r = 0; r < n; ++r)
        for (int32_t e = m.row_ptr[r]; e < m.row_ptr[r + 1]; ++e) {
            const int32_t i = pinv[(size_t)r], k = qinv[(size_t)m.col_idx[e]];
            auto b0 = F.Ti.begin() + F.Tp[(size_t)i], b1 = F.Ti.begin() + F.Tp[(size_t)i + 1];
            auto it = std::lower_bound(b0, b1, k);
            if (it == b1 || *it != k) return nfail(CS_EINVAL, "factor pattern misses an entry of A");
            src[(size_t)(it - F.Ti.begin())] = e;
        }
    std::vector<int32_t> lev((size_t)n, 0), ulev((size_t)n, 0);
    int32_t nl = 0, nu = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t mx = 0;
        for (int32_t p = F.Tp[(size_t)i]; p < F.Tp[(size_t)i + 1]; ++p) {
            const int32_t j = F.Ti[(size_t)p];
            if (j < i) mx = std::max(mx, lev[(size_t)j] + 1);
            else if (j == i) diag[(size_t)i] = p;
        }
        if (diag[(size_t)i] < 0) return nfail(CS_EINVAL, "factor pattern misses a diagonal");
        lev[(size_t)i] = mx;
        nl = std::max(nl, mx + 1);
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t mx = 0;
        for (int32_t p = diag[(size_t)i] + 1; p < F.Tp[(size_t)i + 1]; ++p)
            mx = std::max(mx, ulev[(size_t)F.Ti[(size_t)p]] + 1);
        ulev[(size_t)i] = mx;
        nu = std::max(nu, mx + 1);
    }
    auto group = [n](const std::vector<int32_t> &lv, int32_t nlev, std::vector<int32_t> &ptr) {
        ptr.assign((size_t)nlev + 1, 0);
        for (int32_t i = 0; i < n; ++i) ptr[(size_t)lv[(size_t)i] + 1]++;
        for (int32_t l = 0; l < nlev; ++l) ptr[(size_t)l + 1] += ptr[(size_t)l];
        std::vector<int32_t> rows((size_t)n), fill(ptr.begin(), ptr.end() - 1);
        for (int32_t i = 0; i < n; ++i) rows[(size_t)fill[(size_t)lv[(size_t)i]]++] = i;
        return rows;
    };
    std::vector<int32_t> lrows = group(lev, nl, ns->lptr);
    // The programmed kernel (k_lu_lower_seq) takes every row within its caps, from a
    // static program: per row its header, per L entry (column j) the diagonal position
    // of row j, j and the end of its records, per U(j, k) with k in the row the T
    // position and the row position.  Inside each lower level the programmed rows come
    // first, then rows short enough for the staged kernel, then the rest.  A run of
    // consecutive narrow levels (at most SEQ_LEVEL_ROWS rows, all programmed) is one
    // launch of one wave taking its rows in order; other levels launch one wave per
    // programmed row.
    {
        constexpr int32_t SEQ_LEVEL_ROWS = 2;
        int32_t crow, cl, cu;
        lu_seq_caps(&crow, &cl, &cu);
        std::vector<int32_t> prow, plo, pst;
        auto program = [&](int32_t i, bool emit) {
            const int32_t t0 = F.Tp[(size_t)i], len = F.Tp[(size_t)i + 1] - t0, nlow = diag[(size_t)i] - t0;
            if (len > crow || nlow > cl) return false;
            auto rb = F.Ti.begin() + t0, re = F.Ti.begin() + t0 + len;
            int32_t ne = 0;
            const size_t lb = plo.size() / 3, eb = pst.size() / 2;
            for (int32_t p = t0; p < diag[(size_t)i]; ++p) {
                const int32_t j = F.Ti[(size_t)p];
                for (int32_t q = diag[(size_t)j] + 1; q < F.Tp[(size_t)j + 1]; ++q) {
                    auto it = std::lower_bound(rb + (p - t0) + 1, re, F.Ti[(size_t)q]);
                    if (it == re || *it != F.Ti[(size_t)q]) continue;
                    if (++ne > cu) return false;
                    if (emit) {
                        pst.push_back(q);
                        pst.push_back((int32_t)(it - rb));
                    }
                }
                if (emit) {
                    plo.push_back(diag[(size_t)j]);
                    plo.push_back(j);
                    plo.push_back(ne);
                }
            }
            if (emit) {
                const int32_t h[8] = {i, t0, len, nlow, (int32_t)lb, (int32_t)eb, ne, F.P[(size_t)i]};
                prow.insert(prow.end(), h, h + 8);
            }
            return true;
        };
        std::vector<uint8_t> fit((size_t)n);
        if (!(flags & CS_NEWTON_NO_PROGRAMMED_ROWS))
            for (int32_t i = 0; i < n; ++i) fit[(size_t)i] = program(i, false) ? 1 : 0;
        ns->lfit.assign((size_t)nl, 0);
        ns->lshort.assign((size_t)nl, 0);
        const int32_t cap = lu_stage_entries();
        for (int32_t l = 0; l < nl; ++l) {
            auto b0 = lrows.begin() + ns->lptr[(size_t)l], b1 = lrows.begin() + ns->lptr[(size_t)l + 1];
            auto m1 = std::stable_partition(b0, b1, [&](int32_t i) { return fit[(size_t)i] != 0; });
            auto m2 = std::stable_partition(m1, b1, [&](int32_t i) { return F.Tp[(size_t)i + 1] - F.Tp[(size_t)i] <= cap; });
            ns->lfit[(size_t)l] = (int32_t)(m1 - b0);
            ns->lshort[(size_t)l] = (int32_t)(m2 - m1);
        }
        // connected parts of the L pattern (row i joined to every j with L(i, j) != 0):
        // rows of different parts never wait for each other in the lower solve (the
        // circuits of a batch are such parts)
        std::vector<int32_t> part((size_t)n);
        for (int32_t i = 0; i < n; ++i) part[(size_t)i] = i;
        auto root = [&](int32_t i) {
            while (part[(size_t)i] != i) {
                part[(size_t)i] = part[(size_t)part[(size_t)i]];
                i = part[(size_t)i];
            }
            return i;
        };
        for (int32_t i = 0; i < n; ++i)
            for (int32_t p = F.Tp[(size_t)i]; p < diag[(size_t)i]; ++p) {
                const int32_t a = root(i), c = root(F.Ti[(size_t)p]);
                if (a != c) part[(size_t)std::max(a, c)] = std::min(a, c);
            }
        for (int32_t i = 0; i < n; ++i) part[(size_t)i] = root(i);
        // a level is narrow when every part has at most SEQ_LEVEL_ROWS rows in it and
        // every row is programmed
        std::vector<int32_t> seen((size_t)n, -1), cnt((size_t)n, 0);
        auto narrow = [&](int32_t lv) {
            const int32_t b0 = ns->lptr[(size_t)lv], b1 = ns->lptr[(size_t)lv + 1];
            if (ns->lfit[(size_t)lv] != b1 - b0) return false;
            for (int32_t k = b0; k < b1; ++k) {
                const int32_t pt = part[(size_t)lrows[(size_t)k]];
                if (seen[(size_t)pt] != lv) {
                    seen[(size_t)pt] = lv;
                    cnt[(size_t)pt] = 0;
                }
                if (++cnt[(size_t)pt] > SEQ_LEVEL_ROWS) return false;
            }
            return true;
        };
        std::vector<int32_t> woff;
        for (int32_t l = 0; l < nl;) {
            int32_t e = l;
            while (e < nl && narrow(e)) ++e;
            const int32_t r0 = (int32_t)(prow.size() / 8);
            if (e > l) {
                // the run's rows grouped by part (parts in order of their first row), in
                // level order inside each part: one workgroup per part
                const int32_t k0 = ns->lptr[(size_t)l], k1 = ns->lptr[(size_t)e];
                std::vector<int32_t> rows_run(lrows.begin() + k0, lrows.begin() + k1);
                std::vector<int32_t> parts;
                for (int32_t k = 0; k < k1 - k0; ++k) {
                    const int32_t pt = part[(size_t)rows_run[(size_t)k]];
                    if (std::find(parts.begin(), parts.end(), pt) == parts.end()) parts.push_back(pt);
                }
                std::vector<int32_t> rank((size_t)n, -1);
                for (size_t q = 0; q < parts.size(); ++q) rank[(size_t)parts[q]] = (int32_t)q;
                std::stable_sort(rows_run.begin(), rows_run.end(), [&](int32_t x, int32_t y) {
                    return rank[(size_t)part[(size_t)x]] < rank[(size_t)part[(size_t)y]];
                });
                NewtonState::LStep st{l, e, true, r0, (int32_t)woff.size(), (int32_t)parts.size()};
                int32_t off = 0;
                woff.push_back(0);
                for (size_t q = 0; q < parts.size(); ++q) {
                    while (off < k1 - k0 && part[(size_t)rows_run[(size_t)off]] == parts[q]) ++off;
                    woff.push_back(off);
                }
                ns->lsteps.push_back(st);
                for (int32_t i : rows_run) program(i, true);
                l = e;
            } else {
                ns->lsteps.push_back({l, l + 1, false, r0});
                const int32_t k0 = ns->lptr[(size_t)l];
                for (int32_t k = k0; k < k0 + ns->lfit[(size_t)l]; ++k) program(lrows[(size_t)k], true);
                ++l;
            }
        }
        if (!woff.empty()) NCHECK_HIP(ns->sq_woff.upload(woff), "upload sequential program");
        if (!prow.empty()) {
            NCHECK_HIP(ns->sq_row.upload(prow), "upload sequential program");
            if (!plo.empty()) NCHECK_HIP(ns->sq_lo.upload(plo), "upload sequential program");
            if (!pst.empty()) NCHECK_HIP(ns->sq_st.upload(pst), "upload sequential program");
        }
    }
    // runs of consecutive narrow upper levels (at most lu_upper_seq_rows() rows, each
    // with at most 256 entries right of the diagonal): one workgroup per run
    {
        const int32_t wmax = lu_upper_seq_rows();
        std::vector<int32_t> urows_h = group(ulev, nu, ns->uptr);
        auto narrow = [&](int32_t lv) {
            const int32_t b0 = ns->uptr[(size_t)lv], b1 = ns->uptr[(size_t)lv + 1];
            if (b1 - b0 > wmax) return false;
            for (int32_t k = b0; k < b1; ++k) {
                const int32_t i = urows_h[(size_t)k];
                if (F.Tp[(size_t)i + 1] - diag[(size_t)i] - 1 > 256) return false;
            }
            return true;
        };
        for (int32_t l = 0; l < nu;) {
            int32_t e = l;
            while (e < nu && narrow(e)) ++e;
            if (e - l >= 2 && !(flags & CS_NEWTON_NO_UPPER_RUNS)) {
                ns->usteps.push_back({l, e, true, 0});
                l = e;
            } else {
                ns->usteps.push_back({l, l + 1, false, 0});
                ++l;
            }
        }
        NCHECK_HIP(ns->urows.upload(urows_h), "upload levels");
        NCHECK_HIP(ns->uptr_d.upload(ns->uptr), "upload levels");
    }
    NCHECK_HIP(ns->lrows.upload(lrows), "upload levels");
    NCHECK_HIP(ns->src.upload(src), "upload load map");
    NCHECK_HIP(ns->diag.upload(diag), "upload diagonal positions");
    NCHECK_HIP(ns->y.alloc((size_t)n), "alloc solve vector");
    guard.p = nullptr;
    *out = ns;
    return CS_OK;
}

cs_status ensure_rocsolver(NewtonState &ns, double *A_val, double *b, hipStream_t s) {
    if (ns.rf) return CS_OK;
    if (!ns.handle) NCHECK_RS(rocblas_create_handle(&ns.handle), "rocblas_create_handle");
    NCHECK_RS(rocblas_set_stream(ns.handle, s), "rocblas_set_stream");
    NCHECK_RS(rocsolver_create_rfinfo(&ns.rf, ns.handle), "rocsolver_create_rfinfo");
    NCHECK_RS(rocsolver_dcsrrf_analysis(ns.handle, ns.n, 1, (rocblas_int)ns.nnzA, ns.ptrA.p, ns.indA.p, A_val,
                                        (rocblas_int)ns.nnzT, ns.ptrT.p, ns.indT.p, ns.valT.p, ns.P.p, ns.Q.p, b,
                                        ns.n, ns.rf),
              "rocsolver_dcsrrf_analysis");
    return CS_OK;
}

// The Newton iterations on a built state: stamp() stamps A and b at x.
template <class Stamp>
cs_status newton_loop(NewtonState &ns, Stamp stamp, int32_t solver, double *x, int32_t n_clamp, int32_t max_iter,
                      double vstep, double tol, double *A_val, double *b, int32_t *n_iter, int32_t *converged,
                      double *last_step, double *times_ms, hipStream_t s) {
    const int32_t n = ns.n;
    if (times_ms) times_ms[4] = ns.host_lu_ms;
    const bool lib = solver == CS_SOLVE_ROCSOLVER;
    if (lib) {
        cs_status st = ensure_rocsolver(ns, A_val, b, s);
        if (st != CS_OK) return st;
        NCHECK_RS(rocblas_set_stream(ns.handle, s), "rocblas_set_stream");
    }
    Events ev;
    if (times_ms) {
        for (auto &v : ev.e) NCHECK_HIP(hipEventCreate(&v), "event");
        ev.on = true;
    }
    double step = 0.0;
    for (int32_t it = 1; it <= max_iter; ++it) {
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[0], s), "event");
        cs_status st = stamp();
        if (st != CS_OK) return st;
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[1], s), "event");
        if (lib) {
            NCHECK_RS(rocsolver_dcsrrf_refactlu(ns.handle, n, (rocblas_int)ns.nnzA, ns.ptrA.p, ns.indA.p, A_val,
                                                (rocblas_int)ns.nnzT, ns.ptrT.p, ns.indT.p, ns.valT.p, ns.P.p,
                                                ns.Q.p, ns.rf),
                      "rocsolver_dcsrrf_refactlu");
            if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[2], s), "event");
            NCHECK_RS(rocsolver_dcsrrf_solve(ns.handle, n, 1, (rocblas_int)ns.nnzT, ns.ptrT.p, ns.indT.p,
                                             ns.valT.p, ns.P.p, ns.Q.p, b, n, ns.rf),
                      "rocsolver_dcsrrf_solve");
        } else {
            // refactorisation fused with the forward substitution, level by level
            NCHECK_HIP(launch_lu_load((int32_t)ns.nnzT, ns.src.p, A_val, ns.valT.p, s), "LU load launch");
            for (const auto &step : ns.lsteps) {
                const int32_t *prog = ns.sq_row.p + 8 * (size_t)step.r0;
                if (step.seq) {
                    NCHECK_HIP(launch_lu_lower_seq(step.grid, 0, ns.sq_woff.p + step.w0, prog, ns.sq_lo.p,
                                                   ns.sq_st.p, ns.valT.p, b, ns.y.p, s),
                               "LU lower launch");
                    continue;
                }
                const size_t l = (size_t)step.l0;
                const int32_t nf = ns.lfit[l], nsh = ns.lshort[l];
                const int32_t beg = ns.lptr[l] + nf, cnt = ns.lptr[l + 1] - beg;
                NCHECK_HIP(launch_lu_lower_seq(nf, 1, nullptr, prog, ns.sq_lo.p, ns.sq_st.p, ns.valT.p, b, ns.y.p, s),
                           "LU lower launch");
                NCHECK_HIP(launch_lu_lower_wave(nsh, ns.lrows.p + beg, ns.ptrT.p, ns.indT.p, ns.diag.p, ns.valT.p,
                                                ns.P.p, b, ns.y.p, s),
                           "LU lower launch");
                NCHECK_HIP(launch_lu_lower(cnt - nsh, ns.lrows.p + beg + nsh, ns.ptrT.p, ns.indT.p, ns.diag.p,
                                           ns.valT.p, ns.P.p, b, ns.y.p, s),
                           "LU lower launch");
            }
            if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[2], s), "event");
            for (const auto &step : ns.usteps) {
                const size_t l = (size_t)step.l0;
                if (step.seq)
                    NCHECK_HIP(launch_lu_upper_seq(step.l1 - step.l0, ns.uptr_d.p + l, ns.urows.p, ns.ptrT.p,
                                                   ns.indT.p, ns.diag.p, ns.valT.p, ns.y.p, ns.Q.p, b, s),
                               "LU upper launch");
                else
                    NCHECK_HIP(launch_lu_upper(ns.uptr[l + 1] - ns.uptr[l], ns.urows.p + ns.uptr[l], ns.ptrT.p,
                                               ns.indT.p, ns.diag.p, ns.valT.p, ns.y.p, ns.Q.p, b, s),
                               "LU upper launch");
            }
        }
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[3], s), "event");
        NCHECK_HIP(hipMemsetAsync(ns.step.p, 0, sizeof(unsigned long long), s), "clear step word");
        NCHECK_HIP(launch_newton_update(n, n_clamp, ns.clamp.p, b, x, vstep, ns.step.p, s), "update launch");
        unsigned long long bits = 0;
        NCHECK_HIP(hipMemcpyAsync(&bits, ns.step.p, sizeof(bits), hipMemcpyDeviceToHost, s), "read step");
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[4], s), "event");
        NCHECK_HIP(hipStreamSynchronize(s), "stream synchronise");
        std::memcpy(&step, &bits, sizeof(step));
        if (ev.on)
            for (int k = 0; k < 4; ++k) {
                float ms = 0.0f;
                NCHECK_HIP(hipEventElapsedTime(&ms, ev.e[k], ev.e[k + 1]), "event time");
                times_ms[k] += ms;
            }
        if (n_iter) *n_iter = it;
        if (last_step) *last_step = step;
        if (!std::isfinite(step)) return nfail(CS_EDOMAIN, "Newton step is not finite");
        if (step <= tol) {
            if (converged) *converged = 1;
            return CS_OK;
        }
    }
    return CS_OK;
}

cs_status check_args(double *x, double *A_val, double *b, int32_t solver, int32_t max_iter, double vstep,
                     double tol) {
    if (!x || !A_val || !b) return nfail(CS_EINVAL, "NULL x, A or b");
    if (max_iter < 1 || !(vstep > 0.0) || !(tol >= 0.0)) return nfail(CS_EINVAL, "max_iter >= 1, vstep > 0, tol >= 0");
    if (solver != CS_SOLVE_LEVELS && solver != CS_SOLVE_ROCSOLVER) return nfail(CS_EINVAL, "unknown solver");
    return CS_OK;
}

}  // namespace

cs_status cs_newton(cs_circuit *c, cs_variant variant, int32_t solver, double *x, double ag0, const double *hist,
                    int32_t max_iter, double vstep, double tol, double *A_val, double *b, int32_t *n_iter,
                    int32_t *converged, double *last_step, double *times_ms, void *stream) {
    if (!c) return nfail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return nfail(CS_ESTATE, "cs_build_stamp_map must come first");
    cs_status st = check_args(x, A_val, b, solver, max_iter, vstep, tol);
    if (st != CS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (n_iter) *n_iter = 0;
    if (converged) *converged = 0;
    if (times_ms) std::memset(times_ms, 0, 5 * sizeof(double));
    if (c->h.n_rows == 0) {
        if (converged) *converged = 1;
        if (last_step) *last_step = 0.0;
        return CS_OK;
    }
    if (c->newton && c->newton->device != c->device) {   // the circuit moved to another GPU
        destroy_newton(c->newton);
        c->newton = nullptr;
    }
    auto stamp = [&]() { return cs_eval_stamp(c, variant, x, ag0, hist, A_val, b, stream); };
    if (!c->newton) {
        st = stamp();
        if (st != CS_OK) return st;
        st = build_state(circuit_view(c->h), c->device, A_val, nullptr, c->newton_flags, s, &c->newton);
        if (st != CS_OK) return st;
    }
    return newton_loop(*c->newton, stamp, solver, x, c->h.n_nodes - 1, max_iter, vstep, tol, A_val, b, n_iter,
                       converged, last_step, times_ms, s);
}

cs_status cs_batch_newton(cs_batch *B, int32_t solver, double *x, double ag0, const double *hist, int32_t max_iter,
                          double vstep, double tol, double *A_val, double *b, int32_t *n_iter, int32_t *converged,
                          double *last_step, double *times_ms, void *stream) {
    if (!B) return nfail(CS_EINVAL, "NULL batch");
    cs_status st = check_args(x, A_val, b, solver, max_iter, vstep, tol);
    if (st != CS_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (n_iter) *n_iter = 0;
    if (converged) *converged = 0;
    if (times_ms) std::memset(times_ms, 0, 5 * sizeof(double));
    const size_t nc = B->circ.size();
    const int64_t n_rows = B->row_off[nc];
    if (n_rows == 0) {
        if (converged) *converged = 1;
        if (last_step) *last_step = 0.0;
        return CS_OK;
    }
    if (n_rows >= INDEX_LIMIT || B->nnz_off[nc] >= INDEX_LIMIT) return nfail(CS_ENOTSUP, "batch too large for the solve");
    auto stamp = [&]() { return cs_batch_eval_stamp(B, x, ag0, hist, A_val, b, stream); };
    if (B->newton && B->newton->device != B->device) {
        destroy_newton(B->newton);
        B->newton = nullptr;
    }
    if (!B->newton) {
        st = stamp();   // uploads and plans the batch, then the first values of A
        if (st != CS_OK) return st;
        // the block-diagonal pattern of the batch, its source pairs and clamp flags
        MnaView m;
        std::vector<uint8_t> clamp((size_t)n_rows, 0);
        try {
            B->nt_row_ptr.assign(1, 0);
            B->nt_col_idx.clear();
            for (size_t i = 0; i < nc; ++i) {
                const HostCircuit &h = B->circ[i]->h;
                const int32_t ro = (int32_t)B->row_off[i], zo = (int32_t)B->nnz_off[i];
                for (int32_t r = 0; r < h.n_rows; ++r) B->nt_row_ptr.push_back(zo + h.row_ptr[(size_t)r + 1]);
                for (int32_t cix : h.col_idx) B->nt_col_idx.push_back(ro + cix);
                for (int32_t r = 0; r < h.n_nodes - 1; ++r) clamp[(size_t)ro + r] = 1;
                for (int32_t j = 0; j < h.n_vsrc; ++j) {
                    const int32_t a = h.vsrc[2 * (size_t)j], bb = h.vsrc[2 * (size_t)j + 1];
                    m.src.push_back({a ? ro + a - 1 : -1, bb ? ro + bb - 1 : -1, ro + h.n_nodes - 1 + j});
                }
            }
        } catch (const std::bad_alloc &) {
            return nfail(CS_ENOMEM, "host allocation");
        }
        m.n = (int32_t)n_rows;
        m.row_ptr = B->nt_row_ptr.data();
        m.col_idx = B->nt_col_idx.data();
        st = build_state(m, B->device, A_val, &clamp, 0, s, &B->newton);
        if (st != CS_OK) return st;
    }
    return newton_loop(*B->newton, stamp, solver, x, 0, max_iter, vstep, tol, A_val, b, n_iter, converged, last_step,
                       times_ms, s);
}

cs_status cs_set_newton_options(cs_circuit *c, int32_t flags) {
    if (!c) return nfail(CS_EINVAL, "NULL circuit");
    if (flags & ~(CS_NEWTON_NO_PROGRAMMED_ROWS | CS_NEWTON_NO_UPPER_RUNS)) return nfail(CS_EINVAL, "unknown flag");
    c->newton_flags = flags;
    destroy_newton(c->newton);   // the next cs_newton plans again
    c->newton = nullptr;
    return CS_OK;
}

cs_status cs_factor_host(const cs_circuit *c, const double *A_host, int64_t *nnzT, int32_t *P, int32_t *Q,
                         int32_t *ptrT, int32_t *indT, double *valT) {
    if (!c || !A_host || !nnzT) return nfail(CS_EINVAL, "NULL argument");
    if (!c->h.mapped) return nfail(CS_ESTATE, "cs_build_stamp_map must come first");
    const HostCircuit &h = c->h;
    HostLU F;
    try {
        Err e = factor_mna(circuit_view(h), A_host, F, nullptr);
        if (e.st != CS_OK) return nfail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return nfail(CS_ENOMEM, "host allocation");
    }
    *nnzT = (int64_t)F.Ti.size();
    if (P) std::memcpy(P, F.P.data(), sizeof(int32_t) * F.P.size());
    if (Q) std::memcpy(Q, F.Q.data(), sizeof(int32_t) * F.Q.size());
    if (ptrT) std::memcpy(ptrT, F.Tp.data(), sizeof(int32_t) * F.Tp.size());
    if (indT) std::memcpy(indT, F.Ti.data(), sizeof(int32_t) * F.Ti.size());
    if (valT) std::memcpy(valT, F.Tx.data(), sizeof(double) * F.Tx.size());
    return CS_OK;
}
