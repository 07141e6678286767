/* Oracle elementary functions (test infrastructure; see oracle.h).
 *
 * The stamped values must agree bit for bit between this oracle and the GPU
 * library, so neither side calls a vendor libm for exp/log: both evaluate the
 * same published methods with the same operation order and no contraction.
 *
 *   pexp(a):   Cody & Waite (1980) range reduction, k = rint(a/ln 2),
 *              r = (a - k*LN2_HI) - k*LN2_LO, then the degree-13 Taylor
 *              polynomial of e^r in Horner form, scaled by 2^k (exact).
 *              Used for |a| <= 40.
 *   plog1p(y): log1p(y) = 2*atanh(s), s = y/(2+y) in [0, 1/3] for y in [0, 1];
 *              2*s*P(s^2) with P(z) = sum_{k=0..16} z^k/(2k+1), Horner.
 *   softplus(t) = max(t, 0) + plog1p(pexp(-|t|)); its derivative
 *   sigma(t) = 1/(1+e) for t >= 0 and e/(1+e) otherwise, e = pexp(-|t|).
 *   pcosh(u) = 0.5*(e + 1/e), e = pexp(u).
 *
 * Horner coefficients are formed here at start-up as correctly rounded quotients
 * 1/k! and 1/(2k+1) (k! is exact in binary64 for k <= 18).
 */
#include <complex.h>
#include <math.h>

#include "oracle.h"
#include "oracle_internal.h"

/* RN(1/ln 2); ln 2 truncated to 32 significant bits (so k*LN2_HI is exact for
 * |k| < 2^11); RN(ln 2 - LN2_HI). */
static const double INV_LN2 = 0x1.71547652b82fep+0;
static const double LN2_HI = 0x1.62e42feep-1;
static const double LN2_LO = 0x1.a39ef35793c76p-33;

#define PEXP_DEG 13
#define PLOG_TERMS 17
static double c_exp[PEXP_DEG + 1];
static double c_log[PLOG_TERMS];

__attribute__((constructor)) static void or_init_coeffs(void) {
    double f = 1.0;
    for (int k = 0; k <= PEXP_DEG; ++k) {
        if (k > 0) f = f * (double)k;
        c_exp[k] = 1.0 / f;
    }
    for (int k = 0; k < PLOG_TERMS; ++k) c_log[k] = 1.0 / (double)(2 * k + 1);
}

long long or_opcount_ = 0;
int or_counting_ = 0;
void or_count_ops(int on) { or_counting_ = on; or_opcount_ = 0; }
long long or_ops(void) { return or_opcount_; }
long long or_sizedep_ops_ = 0;
long long or_sizedep_ops(void) { return or_sizedep_ops_; }

double or_pexp(double a) {
    double k = rint(a * INV_LN2);
    double r = (a - k * LN2_HI) - k * LN2_LO;
    double p = c_exp[PEXP_DEG];
    for (int j = PEXP_DEG - 1; j >= 0; --j) p = p * r + c_exp[j];
    OR_COUNT(5 + 2 * PEXP_DEG);
    return ldexp(p, (int)k);
}

double or_plog1p(double y) {
    double s = y / (2.0 + y);
    double z = s * s;
    double p = c_log[PLOG_TERMS - 1];
    for (int j = PLOG_TERMS - 2; j >= 0; --j) p = p * z + c_log[j];
    OR_COUNT(5 + 2 * (PLOG_TERMS - 1));
    return (2.0 * s) * p;
}

double or_softplus(double t) {
    double m = t > 0.0 ? t : 0.0;
    OR_COUNT(1);
    return m + or_plog1p(or_pexp(-fabs(t)));
}

double or_sigma(double t) {
    double e = or_pexp(-fabs(t));
    double d = 1.0 + e;
    OR_COUNT(2);
    return t >= 0.0 ? 1.0 / d : e / d;
}

double or_pcosh(double u) {
    double e = or_pexp(u);
    OR_COUNT(3);
    return 0.5 * (e + 1.0 / e);
}

/* Complex extensions for complex-step differentiation: the same formulas with the
 * branch decisions (k, signs) taken on the real part; 2^k scaling is exact. */
double complex or_cpexp(double complex a) {
    double k = rint(creal(a) * INV_LN2);
    double complex r = (a - k * LN2_HI) - k * LN2_LO;
    double complex p = c_exp[PEXP_DEG];
    for (int j = PEXP_DEG - 1; j >= 0; --j) p = p * r + c_exp[j];
    return p * ldexp(1.0, (int)k);
}

double complex or_cplog1p(double complex y) {
    double complex s = y / (2.0 + y);
    double complex z = s * s;
    double complex p = c_log[PLOG_TERMS - 1];
    for (int j = PLOG_TERMS - 2; j >= 0; --j) p = p * z + c_log[j];
    return (2.0 * s) * p;
}

static double complex cabs_re(double complex t) { return creal(t) >= 0.0 ? t : -t; }

double complex or_csoftplus(double complex t) {
    double complex m = creal(t) > 0.0 ? t : 0.0;
    return m + or_cplog1p(or_cpexp(-cabs_re(t)));
}

double complex or_csigma(double complex t) {
    double complex e = or_cpexp(-cabs_re(t));
    double complex d = 1.0 + e;
    return creal(t) >= 0.0 ? 1.0 / d : e / d;
}

double complex or_cpcosh(double complex u) {
    double complex e = or_cpexp(u);
    return 0.5 * (e + 1.0 / e);
}

/* Vectorised entry for the accuracy checks: kind 0 pexp, 1 plog1p, 2 softplus,
 * 3 sigma, 4 pcosh. */
void or_elem_array(int kind, const double *x, double *y, int64_t n) {
    for (int64_t i = 0; i < n; ++i) {
        switch (kind) {
        case 0: y[i] = or_pexp(x[i]); break;
        case 1: y[i] = or_plog1p(x[i]); break;
        case 2: y[i] = or_softplus(x[i]); break;
        case 3: y[i] = or_sigma(x[i]); break;
        default: y[i] = or_pcosh(x[i]); break;
        }
    }
}
