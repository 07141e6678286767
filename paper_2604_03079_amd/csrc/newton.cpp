// Newton-Raphson loop around the evaluate-and-stamp path: the iteration the paper's
// method serves (Introduction: evaluate the devices at the present point, stamp the
// linearised MNA system, solve it for the next point), with the solve that the paper
// leaves to KLU (Benchmark 2; its Conclusions name the solver as the next
// bottleneck).
//
// Per iteration, on one stream: cs_eval_stamp (any variant), rocSOLVER's sparse LU
// refactorisation of A with the pivots of one host factorisation (sparse_lu.cpp),
// its two triangular solves (b becomes the Newton point y), then k_newton_update:
// d = y - x, node rows clamped to [-vstep, vstep], x += d, and the largest |d|
// read back to decide convergence (max |d| <= tol).
#include <rocsolver/rocsolver.h>

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
    int32_t n = 0;
    int64_t nnzT = 0;
    DevBuf<int32_t> ptrA, indA, ptrT, indT, P, Q;
    DevBuf<double> valT;
    DevBuf<unsigned long long> step;
    rocblas_handle handle = nullptr;
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

// Host factorisation at the values of A (device), upload of the factor pattern and
// the solver's analysis.
cs_status build_state(cs_circuit *c, double *A_val, double *b, hipStream_t s) {
    const HostCircuit &h = c->h;
    const int32_t n = h.n_rows;
    std::vector<double> Ah((size_t)h.nnz);
    NCHECK_HIP(hipMemcpyAsync(Ah.data(), A_val, sizeof(double) * Ah.size(), hipMemcpyDeviceToHost, s), "read A");
    NCHECK_HIP(hipStreamSynchronize(s), "stream synchronise");
    auto t0 = std::chrono::steady_clock::now();
    HostLU F;
    try {
        std::vector<int32_t> Q, pref;
        mna_order(h, Q, pref);
        Err e = host_lu(n, h.row_ptr, h.col_idx, Ah.data(), Q, pref, F);
        if (e.st != CS_OK) return nfail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return nfail(CS_ENOMEM, "host allocation");
    }
    auto ns = new (std::nothrow) NewtonState();
    if (!ns) return nfail(CS_ENOMEM, "host allocation");
    ns->host_lu_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    ns->n = n;
    ns->nnzT = (int64_t)F.Ti.size();
    struct Guard {
        NewtonState *p;
        ~Guard() { delete p; }
    } guard{ns};
    NCHECK_HIP(ns->ptrA.upload(h.row_ptr), "upload pattern");
    NCHECK_HIP(ns->indA.upload(h.col_idx), "upload pattern");
    NCHECK_HIP(ns->ptrT.upload(F.Tp), "upload factor pattern");
    NCHECK_HIP(ns->indT.upload(F.Ti), "upload factor pattern");
    NCHECK_HIP(ns->valT.upload(F.Tx), "upload factors");
    NCHECK_HIP(ns->P.upload(F.P), "upload pivots");
    NCHECK_HIP(ns->Q.upload(F.Q), "upload pivots");
    NCHECK_HIP(ns->step.alloc(1), "alloc step word");
    NCHECK_RS(rocblas_create_handle(&ns->handle), "rocblas_create_handle");
    NCHECK_RS(rocblas_set_stream(ns->handle, s), "rocblas_set_stream");
    NCHECK_RS(rocsolver_create_rfinfo(&ns->rf, ns->handle), "rocsolver_create_rfinfo");
    NCHECK_RS(rocsolver_dcsrrf_analysis(ns->handle, n, 1, (rocblas_int)h.nnz, ns->ptrA.p, ns->indA.p, A_val,
                                        (rocblas_int)ns->nnzT, ns->ptrT.p, ns->indT.p, ns->valT.p, ns->P.p,
                                        ns->Q.p, b, n, ns->rf),
              "rocsolver_dcsrrf_analysis");
    guard.p = nullptr;
    c->newton = ns;
    return CS_OK;
}

}  // namespace

cs_status cs_newton(cs_circuit *c, cs_variant variant, double *x, double ag0, const double *hist, int32_t max_iter,
                    double vstep, double tol, double *A_val, double *b, int32_t *n_iter, int32_t *converged,
                    double *last_step, double *times_ms, void *stream) {
    if (!c) return nfail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return nfail(CS_ESTATE, "cs_build_stamp_map must come first");
    if (!x || !A_val || !b) return nfail(CS_EINVAL, "NULL x, A or b");
    if (max_iter < 1 || !(vstep > 0.0) || !(tol >= 0.0)) return nfail(CS_EINVAL, "max_iter >= 1, vstep > 0, tol >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (n_iter) *n_iter = 0;
    if (converged) *converged = 0;
    if (times_ms) std::memset(times_ms, 0, 5 * sizeof(double));
    const int32_t n = c->h.n_rows;
    if (n == 0) {
        if (converged) *converged = 1;
        if (last_step) *last_step = 0.0;
        return CS_OK;
    }
    if (!c->newton) {
        cs_status st = cs_eval_stamp(c, variant, x, ag0, hist, A_val, b, stream);
        if (st != CS_OK) return st;
        st = build_state(c, A_val, b, s);
        if (st != CS_OK) return st;
    }
    NewtonState &ns = *c->newton;
    if (times_ms) times_ms[4] = ns.host_lu_ms;
    NCHECK_RS(rocblas_set_stream(ns.handle, s), "rocblas_set_stream");
    Events ev;
    if (times_ms) {
        for (auto &v : ev.e) NCHECK_HIP(hipEventCreate(&v), "event");
        ev.on = true;
    }
    const int32_t n_clamp = c->h.n_nodes - 1;
    double step = 0.0;
    for (int32_t it = 1; it <= max_iter; ++it) {
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[0], s), "event");
        cs_status st = cs_eval_stamp(c, variant, x, ag0, hist, A_val, b, stream);
        if (st != CS_OK) return st;
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[1], s), "event");
        NCHECK_RS(rocsolver_dcsrrf_refactlu(ns.handle, n, (rocblas_int)c->h.nnz, ns.ptrA.p, ns.indA.p, A_val,
                                            (rocblas_int)ns.nnzT, ns.ptrT.p, ns.indT.p, ns.valT.p, ns.P.p, ns.Q.p,
                                            ns.rf),
                  "rocsolver_dcsrrf_refactlu");
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[2], s), "event");
        NCHECK_RS(rocsolver_dcsrrf_solve(ns.handle, n, 1, (rocblas_int)ns.nnzT, ns.ptrT.p, ns.indT.p, ns.valT.p,
                                         ns.P.p, ns.Q.p, b, n, ns.rf),
                  "rocsolver_dcsrrf_solve");
        if (ev.on) NCHECK_HIP(hipEventRecord(ev.e[3], s), "event");
        NCHECK_HIP(hipMemsetAsync(ns.step.p, 0, sizeof(unsigned long long), s), "clear step word");
        NCHECK_HIP(launch_newton_update(n, n_clamp, b, x, vstep, ns.step.p, s), "update launch");
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

cs_status cs_factor_host(const cs_circuit *c, const double *A_host, int64_t *nnzT, int32_t *P, int32_t *Q,
                         int32_t *ptrT, int32_t *indT, double *valT) {
    if (!c || !A_host || !nnzT) return nfail(CS_EINVAL, "NULL argument");
    if (!c->h.mapped) return nfail(CS_ESTATE, "cs_build_stamp_map must come first");
    const HostCircuit &h = c->h;
    HostLU F;
    try {
        std::vector<int32_t> q, pref;
        mna_order(h, q, pref);
        Err e = host_lu(h.n_rows, h.row_ptr, h.col_idx, A_host, q, pref, F);
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
