// Adjoint (vector-Jacobian product) of the stamped (A, b) with respect to each
// device's W, L and VTH0.
//
// A and b are sums of per-device contributions, each depending on its own device's
// parameters only, so the gradient of S = <A_bar, A> + <b_bar, b> w.r.t. theta is,
// per device, the derivative of
//   S_dev = sum_{t,u} A_bar[t][u] Y[t][u] + sum_t b_bar[t] b_loc[t]
// over its terminals t, u (cotangents gathered through the device's slot map: no
// colouring, no atomics, every gradient entry has one writer).  With G_t = I_t +
// ag0 Q_t the terminal's current, Y[t][u] = dG_t/dV_u and b_loc[t] = sum_u Y[t][u]
// (V_u - V_s) - G_t + hist_t, so
//   S_dev = sum_t ( D_{U_t} G_t - b_bar[t] G_t ) + const,
//   U_t[u] = A_bar[t][u] + b_bar[t] (V_u - V_s)   (V_s - V_s = 0),
// where D_U is the derivative along the voltage direction U.  Written out over the
// channel's functions, S_dev needs only
//   * Ids and its derivative along U_d - U_s,
//   * hQ (half the inversion charge) and its derivative along U_d + U_s - 2 U_g,
//   * Qb, the overlap charges and the junctions, which depend on the parameters
//     through one per-device constant each (Cg, Cov, Aj) linearly.
// So the adjoint evaluates the channel with two directional partials instead of the
// three voltage partials, and differentiates w.r.t. the parameters in forward mode:
// W and VTH0 act on the nonlinear part only through the threshold constant vth_s,
// L through several constants, so two tangents cover the three parameters, carried
// together in one pass per device (Tan2: the values are computed once):
//   tangent 0: d/dvth_s; dS/dVTH0 = pol dS/dvth_s, and dS/dW adds the linear terms
//              of beta0 (Ids is proportional to it), Cg, Cov and Aj;
//   tangent 1: d/dL through every per-device constant.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>

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

// dS/dAj: the junctions of unit area (their currents, charges and conductances are
// proportional to the area).  The drain-body junction adds J0 = I + ag0 Q at v0 =
// p (V_b - V_d) to G_b and subtracts it from G_d, and dJ0/dV = jy (e_b - e_d).
__device__ __forceinline__ double vjp_junction(const DevCard &cd, double p, const double V[4], double ag0,
                                               const double Yb[16], const double bb[4]) {
    double s = 0.0;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int t = side == 0 ? 0 : 2;   // the diffusion terminal
        double ij, gj, qj, cj;
        junction(cd, 1.0, p * (V[3] - V[t]), ij, gj, qj, cj);
        const double J = p * ij + ag0 * (p * qj);
        const double jy = gj + ag0 * cj;
        const double db = V[3] - V[2], dt = V[t] - V[2];
        // (U_b - U_t)[b] - (U_b - U_t)[t], U_x[u] = A_bar[x][u] + b_bar[x] (V_u - V_s)
        const double Ubb = Yb[12 + 3] + bb[3] * db, Ubt = Yb[12 + t] + bb[3] * dt;
        const double Utb = Yb[t * 4 + 3] + bb[t] * db, Utt = Yb[t * 4 + t] + bb[t] * dt;
        s += jy * ((Ubb - Utb) - (Ubt - Utt)) - (bb[3] - bb[t]) * J;
    }
    return s;
}

// Sensitivities of one device's S_dev: g0, g1 along the two tangents the constants
// k carry (a Tan carries one: g0 = g1), and the value-level factors of the constants
// that enter linearly.
struct VjpParts {
    double g0, g1;  // dS/dtheta through the channel, per tangent
    double s_beta;  // dS/dbeta0
    double s_hq;    // dS/dCg through hQ
    double s_qb;    // dS/dCg through Qb
    double s_cov;   // dS/dCov
    double s_aj;    // dS/dAj (with_junction only)
};

__device__ __forceinline__ double tangent(const Tan2 &x, int i) { return i == 0 ? x.t0 : x.t1; }
__device__ __forceinline__ double tangent(const Tan &x, int) { return x.t; }

template <class T>
__device__ __forceinline__ VjpParts vjp_parts(const DevCard &cd, double p, const DevConstT<T> &k,
                                              const double V[4], double ag0, const double Yb[16],
                                              const double bb[4], bool with_junction) {
    VjpParts r;
    r.s_aj = with_junction ? vjp_junction(cd, p, V, ag0, Yb, bb) : 0.0;
    const double vds = p * (V[0] - V[2]), vgs = p * (V[1] - V[2]), vbs = p * (V[3] - V[2]);
    const bool fwd = vds >= 0.0;
    const double x1 = fwd ? vds : -vds;
    const double x2 = fwd ? vgs : vgs - vds;
    const double x3 = fwd ? vbs : vbs - vds;
    // frame: (x1, x2, x3) = p (V_dr - V_rf, V_g - V_rf, V_b - V_rf), (dr, rf) = (d, s)
    // forward, (s, d) reversed; every index below is static (selects, no arrays
    // indexed by the frame)
    const double dv[4] = {V[0] - V[2], V[1] - V[2], 0.0, V[3] - V[2]};
    double U[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int u = 0; u < 4; ++u) U[t][u] = Yb[t * 4 + u] + bb[t] * dv[u];
    // the frame components of a direction Wv (a 4-vector over d, g, s, b)
    auto frame = [&](const double Wv[4], double out[3]) {
        const double wdr = fwd ? Wv[0] : Wv[2], wrf = fwd ? Wv[2] : Wv[0];
        out[0] = p * (wdr - wrf);
        out[1] = p * (Wv[1] - wrf);
        out[2] = p * (Wv[3] - wrf);
    };
    // U_d - U_s, U_d + U_s - 2 U_g, U_b - U_g, U_dr - U_g, U_rf - U_g
    double UI[4], UQ[4], UB[4], UA[4], US[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        UI[u] = U[0][u] - U[2][u];
        UQ[u] = (U[0][u] + U[2][u]) - 2.0 * U[1][u];
        UB[u] = U[3][u] - U[1][u];
        UA[u] = (fwd ? U[0][u] : U[2][u]) - U[1][u];
        US[u] = (fwd ? U[2][u] : U[0][u]) - U[1][u];
    }
    double wI[3], wQ[3], wB[3], wA[3], wS[3];
    frame(UI, wI);
    frame(UQ, wQ);
    frame(UB, wB);
    frame(UA, wA);
    frame(US, wS);
    const double bdr = fwd ? bb[0] : bb[2], brf = fwd ? bb[2] : bb[0];
    const double cI = bb[0] - bb[2];
    const double cQ = (bb[0] + bb[2]) - 2.0 * bb[1];
    const double cB = bb[3] - bb[1];
    const double sI = fwd ? p : -p, sQ = ag0 * p;   // terminal d carries sI * Ids

    // body bias along x3 (no parameter dependence)
    using D1 = DualN<double, 1>;
    const BodyT<D1> bo = body_bias(cd, D1{x3, {1.0}});
    // Qb = -(Cg k1) sqPs, a function of x3
    r.s_qb = sQ * (-cd.k1) * (bo.sqPs.d[0] * wB[2] - cB * bo.sqPs.v);
    // overlap parts: -Cov (x2 - x1) in the frame's Qd (terminal dr), -Cov x2 in its Qs
    // (terminal rf), both also in Qg = -(Qd + Qs + Qb)
    r.s_cov = -sQ * (((wA[1] - wA[0]) - (bdr - bb[1]) * (x2 - x1)) + (wS[1] - (brf - bb[1]) * x2));
    // Gate part with the partials along x2 and x3.  x1 enters the gate only through
    // the DIBL term -dibl x1 of Vth, next to x2 in Vgst = x2 - Vth, so the gate's
    // x1 partials are dVth/dx1 = -dibl and dVgsteff/dx1 = dibl dVgsteff/dx2.
    using G2 = DualN<T, 2>;
    const G2 X1g{T(x1), {T(0.0), T(0.0)}};
    const G2 X2g{T(x2), {T(1.0), T(0.0)}};
    const G2 Vbg{T(bo.Vbseff.v), {T(0.0), T(bo.Vbseff.d[0])}};
    const G2 sqg{T(bo.sqPs.v), {T(0.0), T(bo.sqPs.d[0])}};
    const GateT<G2> gt = gate(cd, k, X1g, X2g, sqg, Vbg);
    const T vth_x1 = -k.dibl, vg_x1 = k.dibl * gt.Vgsteff.d[0];
    // drain current along U_d - U_s
    using C1 = DualN<T, 1>;
    const C1 X1i{T(x1), {T(wI[0])}};
    const C1 Vthi{gt.Vth.v, {(wI[0] * vth_x1 + wI[1] * gt.Vth.d[0]) + wI[2] * gt.Vth.d[1]}};
    const C1 Vgi{gt.Vgsteff.v, {(wI[0] * vg_x1 + wI[1] * gt.Vgsteff.d[0]) + wI[2] * gt.Vgsteff.d[1]}};
    const C1 Vbi{T(bo.Vbseff.v), {T(wI[2] * bo.Vbseff.d[0])}};
    const C1 sqi{T(bo.sqPs.v), {T(wI[2] * bo.sqPs.d[0])}};
    const C1 Ids = drain_current(cd, k, X1i, Vthi, Vgi, Vbi, bulk_factor(k, sqi));
    // half the inversion charge with d/dx1 on its own (seed 1, as in the stamped
    // model: where the charge smoothing cancels to rounding level in x1 this keeps the
    // rounding of the stamped values' own partials) and the x2-x3 part of
    // U_d + U_s - 2 U_g
    using C2 = DualN<T, 2>;
    const C2 X1q{T(x1), {T(1.0), T(0.0)}};
    const C2 Vgq{gt.Vgsteff.v, {vg_x1, wQ[1] * gt.Vgsteff.d[0] + wQ[2] * gt.Vgsteff.d[1]}};
    const C2 sqq{T(bo.sqPs.v), {T(0.0), T(wQ[2] * bo.sqPs.d[0])}};
    const C2 hQ = half_inversion_charge(cd, k, X1q, Vgq, bulk_factor(k, sqq));
    const T dI = Ids.d[0];
    const T dQ = wQ[0] * hQ.d[0] + hQ.d[1];

    r.g0 = sI * (tangent(dI, 0) - cI * tangent(Ids.v, 0)) + sQ * (tangent(dQ, 0) - cQ * tangent(hQ.v, 0));
    r.g1 = sI * (tangent(dI, 1) - cI * tangent(Ids.v, 1)) + sQ * (tangent(dQ, 1) - cQ * tangent(hQ.v, 1));
    r.s_beta = (sI * (dI.v - cI * Ids.v.v)) / k.beta0.v;
    r.s_hq = (sQ * (dQ.v - cQ * hQ.v.v)) / k.Cg.v;
    return r;
}

// One pass per device, both tangents at once (SPLIT = false), or, for inputs too
// small to give every SIMD several waves, two adjacent lanes per device with one
// tangent each (SPLIT = true: lane 0 of the pair d/dvth_s and the W and VTH0
// gradients, lane 1 d/dL and the L gradient; the same arithmetic per tangent, so the
// same results, with the latency of a lane's chain cut).  The grid is what stays
// resident: a thread takes every (gridDim x blockDim)-th item and loads the next
// one's terminals and parameters while it computes the current one.
template <bool SPLIT>
__global__ void __launch_bounds__(256) k_vjp(KCirc kc, KCall call, const double *A_bar,
                                             const double *b_bar, double *gW, double *gL,
                                             double *gV) {
    constexpr int SH = SPLIT ? 1 : 0;   // items per device: 1 << SH
    const int64_t n_items = (int64_t)kc.n << SH;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    struct Pre {
        int32_t t0, t1, t2, t3, v, isP;
        double W, L, VTH0;
    };
    auto fetch = [&](int64_t item) {
        Pre q{0, 0, 0, 0, 0, 0, 0.0, 0.0, 0.0};
        if (item < n_items) {
            const int ps = (int)(item >> SH);
            const size_t n = (size_t)kc.n;
            q.t0 = kc.term[ps];
            q.t1 = kc.term[n + ps];
            q.t2 = kc.term[2 * n + ps];
            q.t3 = kc.term[3 * n + ps];
            q.v = kc.perm[ps];
            q.isP = kc.pol[ps] < 0 ? 1 : 0;
            q.W = kc.par[ps];
            q.L = kc.par[n + ps];
            q.VTH0 = kc.par[2 * n + ps];
        }
        return q;
    };
    const int64_t first = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Pre nx = fetch(first);
    for (int64_t i = first; i < n_items; i += stride) {
        const Pre cu = nx;
        nx = fetch(i + stride);
        const int pos = (int)(i >> SH);
        const int32_t t0 = cu.t0, t1 = cu.t1, t2 = cu.t2, t3 = cu.t3;
        const int key = pattern_key(t0, t1, t2, t3);
        double Yb[16], bb[4];
        gather_cotangents(key, kc.acode, kc.n, pos, A_bar, b_bar, Yb, bb);
        const double V[4] = {t0 ? call.x[t0 - 1] : 0.0, t1 ? call.x[t1 - 1] : 0.0,
                             t2 ? call.x[t2 - 1] : 0.0, t3 ? call.x[t3 - 1] : 0.0};
        for (;;) {
            const int p0 = __builtin_amdgcn_readfirstlane(cu.isP);
            if (cu.isP == p0) {
                const DevCard &cd = kc.card[p0];
                const double p = p0 ? -1.0 : 1.0;
                // tangent 0: d/dvth_s; tangent 1: d/dL through every constant (W moves
                // vth_s, beta0, Cg, Cov, Aj; L every constant but Cov and Aj)
                const DevConstT<Tan> kl = dev_const(cd, p, Tan(cu.W), Tan(cu.L, 1.0), Tan(cu.VTH0));
                const DevConstW kw = dev_const_dW(cd, cu.W, cu.L);
                // lane of the pair (SPLIT): 0 carries d/dvth_s, 1 carries d/dL
                const bool lt = SPLIT && (i & 1) != 0;
                auto gradW = [&](const VjpParts &r) {
                    double w = kw.vth_s * r.g0 + kw.beta0 * r.s_beta;
                    w += kw.Cg * (r.s_hq + r.s_qb) + kw.Cov * r.s_cov;
                    w += kw.Aj * r.s_aj;
                    gW[cu.v] = w;
                    gV[cu.v] = p * r.g0;
                };
                if constexpr (SPLIT) {
                    auto seed = [&](const Tan &c, double vth) { return Tan(c.v, lt ? c.t : vth); };
                    const DevConstT<Tan> k{seed(kl.vth_s, 1.0), seed(kl.dibl, 0.0), seed(kl.nsce, 0.0),
                                           seed(kl.beta0, 0.0), seed(kl.lambda, 0.0), seed(kl.k1AbL, 0.0),
                                           seed(kl.esatn, 0.0), seed(kl.Cg, 0.0), seed(kl.Cov, 0.0),
                                           seed(kl.Aj, 0.0)};
                    const VjpParts r = vjp_parts(cd, p, k, V, call.ag0, Yb, bb, cd.jmod != 0.0);
                    if (lt) gL[cu.v] = r.g0 + kl.Cg.t * r.s_qb;
                    else gradW(r);
                } else {
                    const DevConstT<Tan2> k{Tan2(kl.vth_s.v, 1.0, kl.vth_s.t), Tan2(kl.dibl.v, 0.0, kl.dibl.t),
                                            Tan2(kl.nsce.v, 0.0, kl.nsce.t), Tan2(kl.beta0.v, 0.0, kl.beta0.t),
                                            Tan2(kl.lambda.v, 0.0, kl.lambda.t), Tan2(kl.k1AbL.v, 0.0, kl.k1AbL.t),
                                            Tan2(kl.esatn.v, 0.0, kl.esatn.t), Tan2(kl.Cg.v, 0.0, kl.Cg.t),
                                            Tan2(kl.Cov.v, 0.0, kl.Cov.t), Tan2(kl.Aj.v, 0.0, kl.Aj.t)};
                    const VjpParts r = vjp_parts(cd, p, k, V, call.ag0, Yb, bb, cd.jmod != 0.0);
                    gradW(r);
                    gL[cu.v] = r.g1 + kl.Cg.t * r.s_qb;
                }
                break;
            }
        }
    }
}

// Compute units and resident blocks per compute unit of the two forms, per device,
// queried on a device's first call (the queries cost host time comparable to the
// kernel on small inputs).  Concurrent first calls store the same values.
namespace {
constexpr int VJP_MAX_DEVICES = 64;
std::atomic<int> g_vjp_cus[VJP_MAX_DEVICES];
std::atomic<int> g_vjp_per[VJP_MAX_DEVICES][2];

hipError_t vjp_launch_facts(int dev, bool split, int *cus, int *per) {
    if (dev >= 0 && dev < VJP_MAX_DEVICES) {
        *cus = g_vjp_cus[dev].load(std::memory_order_relaxed);
        *per = g_vjp_per[dev][split].load(std::memory_order_relaxed);
        if (*cus > 0 && *per > 0) return hipSuccess;
    }
    hipError_t e = hipDeviceGetAttribute(cus, hipDeviceAttributeMultiprocessorCount, dev);
    const void *fn = split ? (const void *)k_vjp<true> : (const void *)k_vjp<false>;
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per, fn, 256, 0);
    if (e == hipSuccess && dev >= 0 && dev < VJP_MAX_DEVICES) {
        g_vjp_cus[dev].store(*cus, std::memory_order_relaxed);
        g_vjp_per[dev][split].store(*per, std::memory_order_relaxed);
    }
    return e;
}
}  // namespace

hipError_t launch_vjp(const KCirc &kc, const KCall &call, const double *A_bar, const double *b_bar,
                      double *gW, double *gL, double *gV, hipStream_t s) {
    if (kc.n == 0) return hipSuccess;
    int dev = 0, cus = 0, per = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    // two lanes per device while the devices fill fewer than one 256-thread block per
    // compute unit, one lane per device beyond (the compute-unit count does not depend
    // on the form: ask with the wider one first)
    if ((e = vjp_launch_facts(dev, false, &cus, &per)) != hipSuccess) return e;
    const bool split = (int64_t)kc.n < (int64_t)cus * 256;
    if (split && (e = vjp_launch_facts(dev, true, &cus, &per)) != hipSuccess) return e;
    const int64_t resident = std::max<int64_t>(1, (int64_t)cus * per);
    const int64_t items = (int64_t)kc.n << (split ? 1 : 0);
    const int grid = (int)std::min<int64_t>((items + 255) / 256, resident);
    if (split) hipLaunchKernelGGL(k_vjp<true>, dim3(grid), dim3(256), 0, s, kc, call, A_bar, b_bar, gW, gL, gV);
    else hipLaunchKernelGGL(k_vjp<false>, dim3(grid), dim3(256), 0, s, kc, call, A_bar, b_bar, gW, gL, gV);
    return hipGetLastError();
}

}  // namespace cs
