// Device model M (BSIM4-core subset) for gfx950, FP64, one device per lane.
//
// The paper evaluates BSIM 4.82 (Methodology, experimental setup) and prints no
// model equations; model M is the project's subset of the published BSIM4 equation
// forms: threshold voltage with body effect, SCE, DIBL and narrow width; unified
// Vgsteff; vertical-field mobility degradation; velocity-saturation Vdsat and the
// smoothed Vdseff; channel-length modulation; charge-conserving inversion/depletion
// charges with a 50/50 partition and overlap charges.
//
// Every operation below is a correctly rounded IEEE binary64 +, -, *, /, sqrt (or an
// exact rint/ldexp/sign change) in a fixed order, with no contraction (the library is
// built with -ffp-contract=off), so a serial CPU evaluation in the same order gives
// the same bits.  Partial derivatives w.r.t. the three frame voltages travel with
// each value ("Dual3"):
//   a*b -> (ab, a_i b + a b_i);  a/b -> r = 1/b, q = a r, q_i = (a_i - q b_i) r;
//   c/b -> r = 1/b, q = c r, q_i = (-(q b_i)) r;  sqrt(a) -> s, h = 0.5/s, s_i = a_i h;
//   exp(a) -> e, e_i = e a_i;  softplus(a) -> sp, sp_i = sigma(a) a_i;
//   c*a scales all four components; a +- c changes the value only;
//   c - a negates the partials.
// One division per quotient: an FP64 division is a multi-instruction sequence on
// gfx950 (reciprocal estimate, Newton steps, scaling and fix-up), a product is one.
#pragma once
#include <hip/hip_runtime.h>

#include "kernel_args.hpp"

namespace cs {

// ---- elementary functions -----------------------------------------------------
// exp: Cody-Waite reduction by ln 2 (k = rint(a/ln 2), ln 2 split into a 32-bit head
// and a correctly rounded tail), degree-13 Taylor polynomial in Horner form with
// coefficients RN(1/j!), exact scaling by 2^k.  Valid for |a| <= 40.
__device__ __forceinline__ double pexp(double a) {
    constexpr double INV_LN2 = 0x1.71547652b82fep+0;
    constexpr double LN2_HI = 0x1.62e42feep-1;
    constexpr double LN2_LO = 0x1.a39ef35793c76p-33;
    const double k = __builtin_rint(a * INV_LN2);
    const double r = (a - k * LN2_HI) - k * LN2_LO;
    double p = 0x1.6124613a86d09p-33;   // 1/13!
    p = p * r + 0x1.1eed8eff8d898p-29;  // 1/12!
    p = p * r + 0x1.ae64567f544e4p-26;  // 1/11!
    p = p * r + 0x1.27e4fb7789f5cp-22;  // 1/10!
    p = p * r + 0x1.71de3a556c734p-19;  // 1/9!
    p = p * r + 0x1.a01a01a01a01ap-16;  // 1/8!
    p = p * r + 0x1.a01a01a01a01ap-13;  // 1/7!
    p = p * r + 0x1.6c16c16c16c17p-10;  // 1/6!
    p = p * r + 0x1.1111111111111p-7;   // 1/5!
    p = p * r + 0x1.5555555555555p-5;   // 1/4!
    p = p * r + 0x1.5555555555555p-3;   // 1/3!
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    return __builtin_ldexp(p, (int)k);
}

// log1p on [0, 1]: 2*atanh(s), s = y/(2+y), series sum_{j<17} s^(2j)/(2j+1), Horner.
__device__ __forceinline__ double plog1p(double y) {
    const double s = y / (2.0 + y);
    const double z = s * s;
    double p = 0x1.f07c1f07c1f08p-6;    // 1/33
    p = p * z + 0x1.0842108421084p-5;   // 1/31
    p = p * z + 0x1.1a7b9611a7b96p-5;   // 1/29
    p = p * z + 0x1.2f684bda12f68p-5;   // 1/27
    p = p * z + 0x1.47ae147ae147bp-5;   // 1/25
    p = p * z + 0x1.642c8590b2164p-5;   // 1/23
    p = p * z + 0x1.8618618618618p-5;   // 1/21
    p = p * z + 0x1.af286bca1af28p-5;   // 1/19
    p = p * z + 0x1.e1e1e1e1e1e1ep-5;   // 1/17
    p = p * z + 0x1.1111111111111p-4;   // 1/15
    p = p * z + 0x1.3b13b13b13b14p-4;   // 1/13
    p = p * z + 0x1.745d1745d1746p-4;   // 1/11
    p = p * z + 0x1.c71c71c71c71cp-4;   // 1/9
    p = p * z + 0x1.2492492492492p-3;   // 1/7
    p = p * z + 0x1.999999999999ap-3;   // 1/5
    p = p * z + 0x1.5555555555555p-2;   // 1/3
    p = p * z + 1.0;
    return (2.0 * s) * p;
}

__device__ __forceinline__ double pcosh(double u) {
    const double e = pexp(u);
    return 0.5 * (e + 1.0 / e);
}

// ---- scalar types ------------------------------------------------------------------
// The model is written once for a scalar type S: plain double (the stamped values,
// bit-exact), Tan, a value with one tangent w.r.t. a device parameter (the
// per-device constants' L-derivatives), or Tan2, a value with two tangents (the
// adjoint's forward-mode pass).  Branches are decided on values.
struct Tan {
    double v, t;
    Tan() = default;
    __device__ __forceinline__ Tan(double x) : v(x), t(0.0) {}
    __device__ __forceinline__ Tan(double x, double dx) : v(x), t(dx) {}
};
__device__ __forceinline__ Tan operator+(Tan a, Tan b) { return {a.v + b.v, a.t + b.t}; }
__device__ __forceinline__ Tan operator-(Tan a, Tan b) { return {a.v - b.v, a.t - b.t}; }
__device__ __forceinline__ Tan operator-(Tan a) { return {-a.v, -a.t}; }
__device__ __forceinline__ Tan operator*(Tan a, Tan b) { return {a.v * b.v, a.t * b.v + a.v * b.t}; }
// Reciprocal and square root for Tan numbers: the hardware estimate refined by two
// Newton steps, within a few ulps of the correctly rounded result (the adjoint's
// values and tangents are checked against the complex-step gradient to a relative
// tolerance, not bit for bit, and never reach the stamped outputs).  The divisors
// and radicands of model M are positive and normal.
__device__ __forceinline__ double rcp_tan(double b) {
    double r = __builtin_amdgcn_rcp(b);
    r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-b, r, 1.0), r, r);
    return r;
}
__device__ __forceinline__ double sqrt_tan(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * y;
    double s = x * y;
    s = __builtin_fma(__builtin_fma(-s, s, x), h, s);
    s = __builtin_fma(__builtin_fma(-s, s, x), h, s);
    return x > 0.0 ? s : 0.0;
}
// Quotients take one reciprocal.
__device__ __forceinline__ Tan operator/(Tan a, Tan b) {
    const double r = rcp_tan(b.v);
    const double q = a.v * r;
    return {q, (a.t - q * b.t) * r};
}
__device__ __forceinline__ Tan operator+(Tan a, double b) { return {a.v + b, a.t}; }
__device__ __forceinline__ Tan operator+(double a, Tan b) { return {a + b.v, b.t}; }
__device__ __forceinline__ Tan operator-(Tan a, double b) { return {a.v - b, a.t}; }
__device__ __forceinline__ Tan operator-(double a, Tan b) { return {a - b.v, -b.t}; }
__device__ __forceinline__ Tan operator*(double a, Tan b) { return {a * b.v, a * b.t}; }
__device__ __forceinline__ Tan operator*(Tan a, double b) { return {a.v * b, a.t * b}; }
__device__ __forceinline__ Tan operator/(Tan a, double b) {
    const double r = rcp_tan(b);
    return {a.v * r, a.t * r};
}
__device__ __forceinline__ Tan operator/(double a, Tan b) {
    const double r = rcp_tan(b.v);
    const double q = a * r;
    return {q, (-(q * b.t)) * r};
}

__device__ __forceinline__ double val(double x) { return x; }
__device__ __forceinline__ double val(const Tan &x) { return x.v; }
__device__ __forceinline__ double gsqrt(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ Tan gsqrt(Tan x) {
    const double s = sqrt_tan(x.v);
    return {s, (0.5 * x.t) * rcp_tan(s)};
}
__device__ __forceinline__ double gabs(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ Tan gabs(Tan x) { return x.v >= 0.0 ? x : -x; }
__device__ __forceinline__ double gexp(double a) { return pexp(a); }
__device__ __forceinline__ Tan gexp(Tan a) {
    const double e = pexp(a.v);
    return {e, e * a.t};
}
__device__ __forceinline__ double glog1p(double y) { return plog1p(y); }
__device__ __forceinline__ Tan glog1p(Tan y) { return {plog1p(y.v), y.t * rcp_tan(1.0 + y.v)}; }
// Value with two tangents (the adjoint carries d/dvth_s and d/dL in one pass); the
// same rules as Tan, each tangent on its own.
struct Tan2 {
    double v, t0, t1;
    Tan2() = default;
    __device__ __forceinline__ Tan2(double x) : v(x), t0(0.0), t1(0.0) {}
    __device__ __forceinline__ Tan2(double x, double a, double b) : v(x), t0(a), t1(b) {}
};
__device__ __forceinline__ Tan2 operator+(Tan2 a, Tan2 b) { return {a.v + b.v, a.t0 + b.t0, a.t1 + b.t1}; }
__device__ __forceinline__ Tan2 operator-(Tan2 a, Tan2 b) { return {a.v - b.v, a.t0 - b.t0, a.t1 - b.t1}; }
__device__ __forceinline__ Tan2 operator-(Tan2 a) { return {-a.v, -a.t0, -a.t1}; }
__device__ __forceinline__ Tan2 operator*(Tan2 a, Tan2 b) {
    return {a.v * b.v, a.t0 * b.v + a.v * b.t0, a.t1 * b.v + a.v * b.t1};
}
__device__ __forceinline__ Tan2 operator/(Tan2 a, Tan2 b) {
    const double r = rcp_tan(b.v);
    const double q = a.v * r;
    return {q, (a.t0 - q * b.t0) * r, (a.t1 - q * b.t1) * r};
}
__device__ __forceinline__ Tan2 operator+(Tan2 a, double b) { return {a.v + b, a.t0, a.t1}; }
__device__ __forceinline__ Tan2 operator+(double a, Tan2 b) { return {a + b.v, b.t0, b.t1}; }
__device__ __forceinline__ Tan2 operator-(Tan2 a, double b) { return {a.v - b, a.t0, a.t1}; }
__device__ __forceinline__ Tan2 operator-(double a, Tan2 b) { return {a - b.v, -b.t0, -b.t1}; }
__device__ __forceinline__ Tan2 operator*(double a, Tan2 b) { return {a * b.v, a * b.t0, a * b.t1}; }
__device__ __forceinline__ Tan2 operator*(Tan2 a, double b) { return {a.v * b, a.t0 * b, a.t1 * b}; }
__device__ __forceinline__ Tan2 operator/(Tan2 a, double b) {
    const double r = rcp_tan(b);
    return {a.v * r, a.t0 * r, a.t1 * r};
}
__device__ __forceinline__ Tan2 operator/(double a, Tan2 b) {
    const double r = rcp_tan(b.v);
    const double q = a * r;
    return {q, (-(q * b.t0)) * r, (-(q * b.t1)) * r};
}
__device__ __forceinline__ double val(const Tan2 &x) { return x.v; }
__device__ __forceinline__ Tan2 gsqrt(Tan2 x) {
    const double s = sqrt_tan(x.v);
    const double h = 0.5 * rcp_tan(s);
    return {s, x.t0 * h, x.t1 * h};
}
__device__ __forceinline__ Tan2 gabs(Tan2 x) { return x.v >= 0.0 ? x : -x; }
__device__ __forceinline__ Tan2 gexp(Tan2 a) {
    const double e = pexp(a.v);
    return {e, e * a.t0, e * a.t1};
}
__device__ __forceinline__ Tan2 glog1p(Tan2 y) {
    const double r = rcp_tan(1.0 + y.v);
    return {plog1p(y.v), y.t0 * r, y.t1 * r};
}
template <class S>
__device__ __forceinline__ S gcosh(S u) {
    const S e = gexp(u);
    return 0.5 * (e + 1.0 / e);
}

// ---- values with three partials -------------------------------------------------
template <class S>
struct Dual3T {
    S v, d0, d1, d2;
};

template <class S>
__device__ __forceinline__ Dual3T<S> seed(double v, int k) {
    return {S(v), S(k == 0 ? 1.0 : 0.0), S(k == 1 ? 1.0 : 0.0), S(k == 2 ? 1.0 : 0.0)};
}
template <class S>
__device__ __forceinline__ Dual3T<S> operator+(Dual3T<S> a, Dual3T<S> b) {
    return {a.v + b.v, a.d0 + b.d0, a.d1 + b.d1, a.d2 + b.d2};
}
template <class S>
__device__ __forceinline__ Dual3T<S> operator-(Dual3T<S> a, Dual3T<S> b) {
    return {a.v - b.v, a.d0 - b.d0, a.d1 - b.d1, a.d2 - b.d2};
}
template <class S>
__device__ __forceinline__ Dual3T<S> operator-(Dual3T<S> a) { return {-a.v, -a.d0, -a.d1, -a.d2}; }
template <class S, class C>
__device__ __forceinline__ Dual3T<S> plus_c(Dual3T<S> a, C c) { return {a.v + c, a.d0, a.d1, a.d2}; }
template <class S, class C>
__device__ __forceinline__ Dual3T<S> minus_c(Dual3T<S> a, C c) { return {a.v - c, a.d0, a.d1, a.d2}; }
template <class S, class C>
__device__ __forceinline__ Dual3T<S> c_minus(C c, Dual3T<S> a) { return {c - a.v, -a.d0, -a.d1, -a.d2}; }
template <class S, class C>
__device__ __forceinline__ Dual3T<S> scale(C c, Dual3T<S> a) {
    return {c * a.v, c * a.d0, c * a.d1, c * a.d2};
}
template <class S>
__device__ __forceinline__ Dual3T<S> operator*(Dual3T<S> a, Dual3T<S> b) {
    return {a.v * b.v, a.d0 * b.v + a.v * b.d0, a.d1 * b.v + a.v * b.d1, a.d2 * b.v + a.v * b.d2};
}
template <class S>
__device__ __forceinline__ Dual3T<S> operator/(Dual3T<S> a, Dual3T<S> b) {
    const S r = 1.0 / b.v;
    const S q = a.v * r;
    return {q, (a.d0 - q * b.d0) * r, (a.d1 - q * b.d1) * r, (a.d2 - q * b.d2) * r};
}
template <class S, class C>
__device__ __forceinline__ Dual3T<S> c_over(C c, Dual3T<S> b) {
    const S r = 1.0 / b.v;
    const S q = c * r;
    return {q, (-(q * b.d0)) * r, (-(q * b.d1)) * r, (-(q * b.d2)) * r};
}
template <class S>
__device__ __forceinline__ Dual3T<S> dsqrt(Dual3T<S> a) {
    const S s = gsqrt(a.v);
    const S h = 0.5 / s;
    return {s, a.d0 * h, a.d1 * h, a.d2 * h};
}
template <class S>
__device__ __forceinline__ Dual3T<S> dexp(Dual3T<S> a) {
    const S e = gexp(a.v);
    return {e, e * a.d0, e * a.d1, e * a.d2};
}
// softplus(t) = max(t, 0) + log1p(e^-|t|); its derivative sigma(t) = 1/(1+e) for
// t >= 0, e/(1+e) otherwise, e = e^-|t|.
template <class S>
__device__ __forceinline__ Dual3T<S> dsoftplus(Dual3T<S> a) {
    const S t = a.v;
    const S e = gexp(-gabs(t));
    const S sp = (val(t) > 0.0 ? t : S(0.0)) + glog1p(e);
    const S dn = 1.0 + e;
    const S sg = val(t) >= 0.0 ? 1.0 / dn : e / dn;
    return {sp, sg * a.d0, sg * a.d1, sg * a.d2};
}

// ---- values with N directional partials --------------------------------------------
// The same rules as Dual3 for N partials, each along a direction chosen by the caller
// (the adjoint carries the partials along the cotangent directions it contracts with).
template <class S, int N>
struct DualN {
    S v;
    S d[N];
};

template <class S, int N>
__device__ __forceinline__ DualN<S, N> operator+(const DualN<S, N> &a, const DualN<S, N> &b) {
    DualN<S, N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
    return r;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> operator-(const DualN<S, N> &a, const DualN<S, N> &b) {
    DualN<S, N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
    return r;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> operator-(const DualN<S, N> &a) {
    DualN<S, N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <class S, int N, class C>
__device__ __forceinline__ DualN<S, N> plus_c(DualN<S, N> a, C c) {
    a.v = a.v + c;
    return a;
}
template <class S, int N, class C>
__device__ __forceinline__ DualN<S, N> minus_c(DualN<S, N> a, C c) {
    a.v = a.v - c;
    return a;
}
template <class S, int N, class C>
__device__ __forceinline__ DualN<S, N> c_minus(C c, const DualN<S, N> &a) {
    DualN<S, N> r;
    r.v = c - a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
    return r;
}
template <class S, int N, class C>
__device__ __forceinline__ DualN<S, N> scale(C c, const DualN<S, N> &a) {
    DualN<S, N> r;
    r.v = c * a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = c * a.d[i];
    return r;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> operator*(const DualN<S, N> &a, const DualN<S, N> &b) {
    DualN<S, N> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
    return r;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> operator/(const DualN<S, N> &a, const DualN<S, N> &b) {
    const S r = 1.0 / b.v;
    DualN<S, N> o;
    o.v = a.v * r;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = (a.d[i] - o.v * b.d[i]) * r;
    return o;
}
template <class S, int N, class C>
__device__ __forceinline__ DualN<S, N> c_over(C c, const DualN<S, N> &b) {
    const S r = 1.0 / b.v;
    DualN<S, N> o;
    o.v = c * r;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = (-(o.v * b.d[i])) * r;
    return o;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> dsqrt(const DualN<S, N> &a) {
    DualN<S, N> o;
    o.v = gsqrt(a.v);
    const S h = 0.5 / o.v;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = a.d[i] * h;
    return o;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> dexp(const DualN<S, N> &a) {
    DualN<S, N> o;
    o.v = gexp(a.v);
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = o.v * a.d[i];
    return o;
}
template <class S, int N>
__device__ __forceinline__ DualN<S, N> dsoftplus(const DualN<S, N> &a) {
    const S t = a.v;
    const S e = gexp(-gabs(t));
    DualN<S, N> o;
    o.v = (val(t) > 0.0 ? t : S(0.0)) + glog1p(e);
    const S dn = 1.0 + e;
    const S sg = val(t) >= 0.0 ? 1.0 / dn : e / dn;
#pragma unroll
    for (int i = 0; i < N; ++i) o.d[i] = sg * a.d[i];
    return o;
}

// Size-dependent constants of one device (depend on W, L, VTH0 only).
template <class S>
struct SizeDepT {
    S Leff, vth_s, theta_dibl, theta_sce, beta0, lambda, AbL, Cg, Cov, Aj;
};

template <class S>
__device__ __forceinline__ SizeDepT<S> size_dep(const DevCard &cd, double pol, S W, S L, S VTH0) {
    SizeDepT<S> s;
    const S Weff = W - cd.TWO_WINT;
    s.Leff = L - cd.TWO_LINT;
    const S VTH0i = pol * VTH0;
    s.theta_sce = 0.5 / (gcosh((cd.dvt1 * s.Leff) / cd.LT) - 1.0);
    s.theta_dibl = 0.5 / (gcosh((cd.dsub * s.Leff) / cd.LT) - 1.0);
    s.vth_s = (VTH0i - (cd.dvt0 * s.theta_sce) * cd.VBI_M_PHIS) + cd.K3_TOXE_PHIS / (Weff + cd.w0);
    s.beta0 = (Weff * cd.COXE) / s.Leff;
    s.lambda = cd.lambda_l / s.Leff;
    s.AbL = (cd.a0 * s.Leff) / (s.Leff + cd.LA);
    s.Cg = (Weff * s.Leff) * cd.COXE;
    s.Cov = cd.cgdo * Weff;
    s.Aj = Weff * cd.hdif;   // junction area
    return s;
}

// The per-device constants the bias-dependent part reads, as the products it uses
// (the same operations, in the same order, as written inline in the model): they
// depend on W, L, VTH0 and the card only, so they are computed once per parameter
// set, not per Newton iteration.  Field order = row order of KCirc::sdp.
template <class S>
struct DevConstT {
    S vth_s, dibl, nsce, beta0, lambda, k1AbL, esatn, Cg, Cov, Aj;
};
static_assert(sizeof(DevConstT<double>) == NSD * sizeof(double), "one row per field");

template <class S>
__device__ __forceinline__ DevConstT<S> dev_const(const DevCard &cd, double pol, S W, S L, S VTH0) {
    const SizeDepT<S> sd = size_dep(cd, pol, W, L, VTH0);
    DevConstT<S> k;
    k.vth_s = sd.vth_s;
    k.dibl = cd.eta0 * sd.theta_dibl;                   // DIBL coefficient of M3
    k.nsce = (cd.cdsc * sd.theta_sce) / cd.COXE;        // SCE term of M4
    k.beta0 = sd.beta0;
    k.lambda = sd.lambda;
    k.k1AbL = cd.k1 * sd.AbL;                           // numerator of M8's Abulk term
    k.esatn = cd.TWO_VSAT * sd.Leff;                    // numerator of M8's EsatL
    k.Cg = sd.Cg;
    k.Cov = sd.Cov;
    k.Aj = sd.Aj;
    return k;
}

// d/dW of the per-device constants that depend on W (vth_s through the narrow-width
// term, beta0, Cg, Cov, Aj); the others depend on L and the card only.
struct DevConstW {
    double vth_s, beta0, Cg, Cov, Aj;
};
__device__ __forceinline__ DevConstW dev_const_dW(const DevCard &cd, double W, double L) {
    const double Weff = W - cd.TWO_WINT;
    const double Leff = L - cd.TWO_LINT;
    const double ww = Weff + cd.w0;
    return {-cd.K3_TOXE_PHIS / (ww * ww), cd.COXE / Leff, Leff * cd.COXE, cd.cgdo, cd.hdif};
}

// One source/drain-body junction of forward voltage v (body above the diffusion for
// NMOS) and area A: diode current Ij and conductance gj (exponent clamped at -40,
// tangent continuation above vjmax), abrupt-junction depletion charge Qj and
// capacitance Cj (linear-capacitance continuation above fc pb).  The exponentials
// and roots depend on v only; A carries the parameter sensitivity.
template <class S>
__device__ __forceinline__ void junction(const DevCard &cd, S A, double v, S &Ij, S &gj, S &Qj, S &Cj) {
    const S Is = cd.js * A;
    if (v <= cd.vjmax) {
        const double a = v / cd.NJ_VT;
        const double e = pexp(a > -40.0 ? a : -40.0);
        Ij = Is * (e - 1.0);
        gj = (Is * e) / cd.NJ_VT;
    } else {
        const double el = pexp(cd.vjmax / cd.NJ_VT);
        const S gl = (Is * el) / cd.NJ_VT;
        Ij = Is * (el - 1.0) + gl * (v - cd.vjmax);
        gj = gl;
    }
    const S Cj0 = cd.cj * A;
    if (v < cd.FCPB) {
        const double r = __builtin_sqrt(1.0 - v / cd.pb);
        Qj = (Cj0 * cd.TWO_PB) * (1.0 - r);
        Cj = Cj0 / r;
    } else {
        Qj = Cj0 * (cd.JF1 + ((cd.JF3 * (v - cd.FCPB)) + cd.QUARTER_PB * ((v * v) - cd.FCPB2)) / cd.JF2);
        Cj = (Cj0 / cd.JF2) * (cd.JF3 + 0.5 * (v / cd.pb));
    }
}

// Effective body bias and sqrt(phis - Vbseff): functions of the frame's x3 alone.
template <class D>
struct BodyT {
    D Vbseff, sqPs;
};
template <class D>
__device__ __forceinline__ BodyT<D> body_bias(const DevCard &cd, const D &X3) {
    const D T0 = minus_c(c_minus(cd.VBM, X3), cd.delta1);
    const D sq0 = dsqrt(plus_c(T0 * T0, cd.FOUR_DELTA1_VBM));
    const D Vbseff = c_minus(cd.VBM, scale(0.5, T0 + sq0));
    const D sqPs = dsqrt(c_minus(cd.phis, Vbseff));
    return {Vbseff, sqPs};
}

// The channel of model M in the frame (x1, x2, x3) = (|vds|, gate, body voltages
// from the source side), in four parts, each generic over the number type D (value
// with partials) and the per-device constants K (fields of one scalar type): the
// gate part (threshold and effective overdrive), the bulk-charge factor, the drain
// current and half the inversion charge (the 50/50 partition).
template <class D>
struct GateT {
    D Vth, Vgsteff;
};
template <class D, class K>
__device__ __forceinline__ GateT<D> gate(const DevCard &cd, const K &sd, const D &X1, const D &X2,
                                         const D &sqPs, const D &Vbseff) {
    // threshold voltage
    const D Vth = (plus_c(scale(cd.k1, minus_c(sqPs, cd.SQPHIS)), sd.vth_s) - scale(cd.k2, Vbseff))
                  - scale(sd.dibl, X1);
    // subthreshold swing factor
    // (the constant factors of the Cdep term are the card constant NCDEP)
    const D n = plus_c(plus_c(c_over(cd.NCDEP, sqPs), 1.0), sd.nsce);
    const D nvt = scale(cd.VT, n);
    const D Vgst = X2 - Vth;
    // unified effective gate overdrive
    const D h = scale(0.5, Vgst);
    const D num6 = nvt * dsoftplus(h / nvt);
    const D ex6 = dexp((-minus_c(h, cd.voff)) / nvt);
    const D den6 = plus_c(scale(cd.COXE_KS, n) * ex6, 0.5);
    const D Vgsteff = num6 / den6;
    return {Vth, Vgsteff};
}
template <class D, class K>
__device__ __forceinline__ D bulk_factor(const K &sd, const D &sqPs) {
    return plus_c(c_over(sd.k1AbL, scale(2.0, sqPs)), 1.0);
}
template <class D, class K>
__device__ __forceinline__ D drain_current(const DevCard &cd, const K &sd, const D &X1, const D &Vth,
                                           const D &Vgsteff, const D &Vbseff, const D &Abulk) {
    // mobility
    const D Ee = scale(cd.INV_TOXE, Vgsteff + scale(2.0, Vth));
    const D mden = plus_c(plus_c(scale(cd.uc, Vbseff), cd.ua) * Ee, 1.0) + scale(cd.ub, Ee * Ee);
    const D mu = c_over(cd.u0, mden);
    // saturation
    const D EsatL = c_over(sd.esatn, mu);
    const D V2 = plus_c(Vgsteff, cd.TWO_VT);
    const D Vdsat = (EsatL * V2) / ((Abulk * EsatL) + V2);
    const D T1 = minus_c(Vdsat - X1, cd.delta);
    const D sq1 = dsqrt((T1 * T1) + scale(cd.FOUR_DELTA, Vdsat));
    const D Vdseff = Vdsat - scale(0.5, T1 + sq1);
    // drain current with channel-length modulation
    const D c11 = (scale(sd.beta0, mu) * Vgsteff) * Vdseff;
    const D f11 = c_minus(1.0, (Abulk * Vdseff) / scale(2.0, V2));
    const D g11 = plus_c(Vdseff / EsatL, 1.0);
    const D Ids0 = (c11 * f11) / g11;
    return Ids0 * plus_c(scale(sd.lambda, X1 - Vdseff), 1.0);
}
template <class D, class K>
__device__ __forceinline__ D half_inversion_charge(const DevCard &cd, const K &sd, const D &X1,
                                                   const D &Vgsteff, const D &Abulk) {
    const D Vdc = Vgsteff / Abulk;
    const D T2 = minus_c(Vdc - X1, cd.delta);
    const D sq2 = dsqrt((T2 * T2) + scale(cd.FOUR_DELTA, Vdc));
    const D Vdcv = Vdc - scale(0.5, T2 + sq2);
    const D AV = Abulk * Vdcv;
    const D Tq = Vgsteff - scale(0.5, AV);
    const D Qinv = scale(-sd.Cg, Tq + (AV * AV) / scale(12.0, Tq));
    return scale(0.5, Qinv);
}

// The whole channel with one number type: drain current Ids, half the inversion
// charge hQ and the depletion charge Qb.
template <class D>
struct ChannelT {
    D Ids, hQ, Qb;
};
template <class D, class K>
__device__ __forceinline__ ChannelT<D> channel(const DevCard &cd, const K &sd, const D &X1, const D &X2,
                                               const D &Vbseff, const D &sqPs) {
    const GateT<D> g = gate(cd, sd, X1, X2, sqPs, Vbseff);
    const D Abulk = bulk_factor(sd, sqPs);
    const D Ids = drain_current(cd, sd, X1, g.Vth, g.Vgsteff, Vbseff, Abulk);
    const D hQ = half_inversion_charge(cd, sd, X1, g.Vgsteff, Abulk);
    const D Qb = scale(-(sd.Cg * cd.k1), sqPs);
    return {Ids, hQ, Qb};
}

// Local outputs of one device: the 9 independent entries of Y (rows/cols d, g, b;
// the s row and column follow from conservation) and the local RHS.
template <class S>
struct DevOutT {
    S Ydd, Ydg, Ydb, Ygd, Ygg, Ygb, Ybd, Ybg, Ybb;
    S bd, bg, bs, bb;
};

// Model M at terminal voltages V = (Vd, Vg, Vs, Vb).  qout (optional): the terminal
// charges (d, g, s, b) at V, for the history term of the next integration step.
// J = false compiles the junction terms out (cards with jmod = 0 only).
template <class S, bool J = true>
__device__ __forceinline__ DevOutT<S> eval_model(const DevCard &cd, double p, const DevConstT<S> &sd,
                                                 double Vd, double Vg, double Vs, double Vb,
                                                 double ag0, const double *hist, double *qout = nullptr) {
    using D = Dual3T<S>;
    const double vds = p * (Vd - Vs), vgs = p * (Vg - Vs), vbs = p * (Vb - Vs);
    const bool fwd = vds >= 0.0;
    const double x1 = fwd ? vds : -vds;
    const double x2 = fwd ? vgs : vgs - vds;
    const double x3 = fwd ? vbs : vbs - vds;
    const D X1 = seed<S>(x1, 0), X2 = seed<S>(x2, 1), X3 = seed<S>(x3, 2);

    const BodyT<D> bo = body_bias(cd, X3);
    const ChannelT<D> ch = channel(cd, sd, X1, X2, bo.Vbseff, bo.sqPs);
    const D &Ids = ch.Ids;
    const D &hQ = ch.hQ;
    const D &Qb = ch.Qb;
    const D Qd = hQ - scale(sd.Cov, X2 - X1);
    const D Qs = hQ - scale(sd.Cov, X2);
    const D Qg = -((Qd + Qs) + Qb);

    // frame partials -> partials w.r.t. (vds, vgs, vbs); reverse mode swaps d and s
    auto term = [&](const D &f, S &gd, S &gg, S &gb) {
        if (fwd) { gd = f.d0; gg = f.d1; gb = f.d2; }
        else { gd = ((-f.d0) - f.d1) - f.d2; gg = f.d1; gb = f.d2; }
    };
    S iD, iG, iB, qdD, qdG, qdB, qsD, qsG, qsB, qgD, qgG, qgB, qbD, qbG, qbB;
    term(Ids, iD, iG, iB);
    term(Qd, qdD, qdG, qdB);
    term(Qs, qsD, qsG, qsB);
    term(Qg, qgD, qgG, qgB);
    term(Qb, qbD, qbG, qbB);
    S Idp, Qdp, Qsp;
    if (fwd) {
        Idp = Ids.v; Qdp = Qd.v; Qsp = Qs.v;
    } else {
        Idp = -Ids.v; Qdp = Qs.v; Qsp = Qd.v;
        iD = -iD; iG = -iG; iB = -iB;
        S t;
        t = qdD; qdD = qsD; qsD = t;
        t = qdG; qdG = qsG; qsG = t;
        t = qdB; qdB = qsB; qsB = t;
    }
    (void)qsD; (void)qsG; (void)qsB;

    // junctions (card jmod): drain-body then source-body, current and charge from
    // the body terminal to the diffusion terminal; jy = g + ag0 C
    const bool jon = J && cd.jmod != 0.0;
    S jI0 = 0.0, jI1 = 0.0, jQ0 = 0.0, jQ1 = 0.0, jy0 = 0.0, jy1 = 0.0;
    if (jon) {
        S ij, gj, qj, cj;
        junction(cd, sd.Aj, p * (Vb - Vd), ij, gj, qj, cj);
        jI0 = p * ij; jQ0 = p * qj; jy0 = gj + ag0 * cj;
        junction(cd, sd.Aj, p * (Vb - Vs), ij, gj, qj, cj);
        jI1 = p * ij; jQ1 = p * qj; jy1 = gj + ag0 * cj;
    }

    DevOutT<S> o;
    o.Ydd = iD + ag0 * qdD; o.Ydg = iG + ag0 * qdG; o.Ydb = iB + ag0 * qdB;
    o.Ygd = ag0 * qgD;      o.Ygg = ag0 * qgG;      o.Ygb = ag0 * qgB;
    o.Ybd = ag0 * qbD;      o.Ybg = ag0 * qbG;      o.Ybb = ag0 * qbB;
    if (jon) {
        o.Ydd = o.Ydd + jy0;
        o.Ybd = o.Ybd - jy0;
        o.Ydb = o.Ydb - jy0;
        o.Ybb = (o.Ybb + jy0) + jy1;
    }
    const S Ysd = -((o.Ydd + o.Ygd) + o.Ybd);
    const S Ysg = -((o.Ydg + o.Ygg) + o.Ybg);
    const S Ysb = -((o.Ydb + o.Ygb) + o.Ybb);

    // physical terminal currents and charges
    S I_d = p * Idp, I_s = p * (-Idp), I_b = 0.0;
    S Q_d = p * Qdp, Q_g = p * Qg.v, Q_s = p * Qsp, Q_b = p * Qb.v;
    if (jon) {
        I_d = I_d - jI0; I_s = I_s - jI1; I_b = jI0 + jI1;
        Q_d = Q_d - jQ0; Q_s = Q_s - jQ1; Q_b = (Q_b + jQ0) + jQ1;
    }
    if (qout) {
        qout[0] = val(Q_d);
        qout[1] = val(Q_g);
        qout[2] = val(Q_s);
        qout[3] = val(Q_b);
    }
    const double dvd = Vd - Vs, dvg = Vg - Vs, dvb = Vb - Vs;
    o.bd = (((o.Ydd * dvd + o.Ydg * dvg) + o.Ydb * dvb) - I_d) - ag0 * Q_d;
    o.bg = (((o.Ygd * dvd + o.Ygg * dvg) + o.Ygb * dvb) - 0.0) - ag0 * Q_g;
    o.bs = (((Ysd * dvd + Ysg * dvg) + Ysb * dvb) - I_s) - ag0 * Q_s;
    o.bb = (((o.Ybd * dvd + o.Ybg * dvg) + o.Ybb * dvb) - I_b) - ag0 * Q_b;
    if (hist) {
        o.bd = o.bd + hist[0];
        o.bg = o.bg + hist[1];
        o.bs = o.bs + hist[2];
        o.bb = o.bb + hist[3];
    }
    return o;
}

// The full local matrix, rows and columns (d, g, s, b), in the same order of
// operations the conservation rules define.
template <class S>
__device__ __forceinline__ void full_Y(const DevOutT<S> &o, S Y[16]) {
    Y[0] = o.Ydd; Y[1] = o.Ydg; Y[3] = o.Ydb;
    Y[4] = o.Ygd; Y[5] = o.Ygg; Y[7] = o.Ygb;
    Y[12] = o.Ybd; Y[13] = o.Ybg; Y[15] = o.Ybb;
    Y[8] = -((o.Ydd + o.Ygd) + o.Ybd);
    Y[9] = -((o.Ydg + o.Ygg) + o.Ybg);
    Y[11] = -((o.Ydb + o.Ygb) + o.Ybb);
    Y[2] = -((Y[0] + Y[1]) + Y[3]);
    Y[6] = -((Y[4] + Y[5]) + Y[7]);
    Y[10] = -((Y[8] + Y[9]) + Y[11]);
    Y[14] = -((Y[12] + Y[13]) + Y[15]);
}

using Dual3 = Dual3T<double>;
using SizeDep = SizeDepT<double>;
using DevOut = DevOutT<double>;

}  // namespace cs
