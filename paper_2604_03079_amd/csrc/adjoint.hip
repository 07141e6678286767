// Adjoint (vector-Jacobian product) of the stamped (A, b) with respect to each
// device's W, L and VTH0.
//
// A and b are sums of per-device contributions, each depending on its own device's
// parameters only, so the gradient of <A_bar, A> + <b_bar, b> w.r.t. theta_k is
//   sum_{(t,u)} A_bar[slot(t,u)] dY_k[t][u]/dtheta_k + sum_t b_bar[row(t)] dbl_k[t]/dtheta_k
// over the device's non-ground terminals.  The cotangents are gathered through the
// device's slot map (no colouring, no atomics: every gradient entry has one writer),
// and a forward-mode sweep of the model per parameter (the tangent of W, L or VTH0
// carried alongside every value and partial) recomputes the intermediates instead
// of storing them.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernel_args.hpp"
#include "launch.hpp"
#include "model.hpp"
#include "stamp.hpp"

namespace cs {

template <int KEY>
__device__ __forceinline__ void gather_pattern(const int32_t *acode, int n, int pos,
                                               const double *A_bar, const double *b_bar,
                                               double Yb[16], double bb[4]) {
    if constexpr (Pat<KEY>::valid()) {
        constexpr int K = Pat<KEY>::k();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                constexpr int dummy = 0;
                (void)dummy;
                const int it = Pat<KEY>::idx(t), iu = Pat<KEY>::idx(u);
                Yb[t * 4 + u] = (it >= 0 && iu >= 0) ? A_bar[acode[(size_t)(it * K + iu) * n + pos]] : 0.0;
            }
            const int it = Pat<KEY>::idx(t);
            bb[t] = it >= 0 ? b_bar[acode[(size_t)(K * K + it) * n + pos]] : 0.0;
        }
    }
}

__device__ __forceinline__ void gather_cotangents(int key, const int32_t *acode, int n, int pos,
                                                  const double *A_bar, const double *b_bar,
                                                  double Yb[16], double bb[4]) {
    for (;;) {
        const int k0 = __builtin_amdgcn_readfirstlane(key);
        if (key == k0) {
            switch (k0) {
#define CS_G(q) case q: gather_pattern<q>(acode, n, pos, A_bar, b_bar, Yb, bb); break;
#define CS_G10(q) CS_G(q) CS_G(q + 1) CS_G(q + 2) CS_G(q + 3) CS_G(q + 4) CS_G(q + 5) \
    CS_G(q + 6) CS_G(q + 7) CS_G(q + 8) CS_G(q + 9)
                CS_G10(0) CS_G10(10) CS_G10(20) CS_G10(30) CS_G10(40) CS_G10(50)
                CS_G10(60) CS_G10(70) CS_G10(80) CS_G10(90) CS_G10(100) CS_G10(110)
#undef CS_G10
#undef CS_G
                default: break;
            }
            break;
        }
    }
}

// One (device, parameter) pair per thread: thread i takes parameter dir = i / n of
// device position i % n, so the three forward-mode sweeps of a device run in three
// lanes at once (a wave holds one parameter and consecutive devices).
__global__ void __launch_bounds__(256) k_vjp(KCirc kc, KCall call, const double *A_bar,
                                             const double *b_bar, double *gW, double *gL,
                                             double *gV) {
    const int64_t total = 3 * (int64_t)kc.n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int dir = (int)(i / kc.n);
        const int pos = (int)(i - (int64_t)dir * kc.n);
        const int32_t t0 = kc.term[pos], t1 = kc.term[(size_t)kc.n + pos];
        const int32_t t2 = kc.term[2 * (size_t)kc.n + pos], t3 = kc.term[3 * (size_t)kc.n + pos];
        const int key = pattern_key(t0, t1, t2, t3);
        double Yb[16], bb[4];
        gather_cotangents(key, kc.acode, kc.n, pos, A_bar, b_bar, Yb, bb);
        const double W = kc.par[pos];
        const double L = kc.par[(size_t)kc.n + pos];
        const double VTH0 = kc.par[2 * (size_t)kc.n + pos];
        const double Vd = t0 ? call.x[t0 - 1] : 0.0, Vg = t1 ? call.x[t1 - 1] : 0.0;
        const double Vs = t2 ? call.x[t2 - 1] : 0.0, Vb = t3 ? call.x[t3 - 1] : 0.0;
        const int32_t v = kc.perm[pos];
        const double *hist = call.hist ? call.hist + 4 * (size_t)v : nullptr;
        const int isP = kc.pol[pos] < 0 ? 1 : 0;
        double g = 0.0;
        for (;;) {
            const int p0 = __builtin_amdgcn_readfirstlane(isP);
            if (isP == p0) {
                const DevCard &cd = kc.card[p0];
                const double p = p0 ? -1.0 : 1.0;
                const Tan Wt(W, dir == 0 ? 1.0 : 0.0), Lt(L, dir == 1 ? 1.0 : 0.0);
                const Tan Vt(VTH0, dir == 2 ? 1.0 : 0.0);
                const DevConstT<Tan> k = dev_const(cd, p, Wt, Lt, Vt);
                const DevOutT<Tan> o = eval_model(cd, p, k, Vd, Vg, Vs, Vb, call.ag0, hist);
                Tan Y[16];
                full_Y(o, Y);
                double acc = 0.0;
#pragma unroll
                for (int k = 0; k < 16; ++k) acc += Yb[k] * Y[k].t;
                acc += bb[0] * o.bd.t + bb[1] * o.bg.t + bb[2] * o.bs.t + bb[3] * o.bb.t;
                g = acc;
                break;
            }
        }
        (dir == 0 ? gW : dir == 1 ? gL : gV)[v] = g;
    }
}

hipError_t launch_vjp(const KCirc &kc, const KCall &call, const double *A_bar, const double *b_bar,
                      double *gW, double *gL, double *gV, hipStream_t s) {
    if (kc.n == 0) return hipSuccess;
    const int64_t total = 3 * (int64_t)kc.n;
    const int grid = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_vjp, dim3(grid), dim3(256), 0, s, kc, call, A_bar, b_bar, gW, gL, gV);
    return hipGetLastError();
}

}  // namespace cs
