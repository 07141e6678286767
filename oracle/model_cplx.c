/* Complex instantiation of model M for complex-step differentiation
 * (Squire & Trapp 1998; Martins, Sturdza & Alonso 2003): a parameter theta is
 * evaluated at theta + i*h and d(output)/d(theta) = Im(output)/h, free of
 * subtractive cancellation.  Branches are taken on real parts. */
#include <complex.h>
#include <math.h>

#include "oracle.h"
#include "oracle_internal.h"

#define T double complex
#define FN(name) name##_cx
#define S_SQRT csqrt
#define S_PEXP or_cpexp
#define S_SOFTPLUS or_csoftplus
#define S_SIGMA or_csigma
#define S_PCOSH or_cpcosh
#define S_PLOG1P or_cplog1p
#define S_RE(x) creal(x)
#define CNT(n) ((void)0)
#define SIZEDEP_BEGIN ((void)0)
#define SIZEDEP_END ((void)0)
#define WITH_TRACE 0
#include "model_m.inc"

void or_device_eval_c(const or_card *card, int pol, double complex W, double complex L,
                      double complex VTH0, const double V[4], double ag0, const double *hist,
                      double complex Y[16], double complex bl[4], double complex Icur[4],
                      double complex Q[4]) {
    or_device_eval_cx(card, pol, W, L, VTH0, V, ag0, hist, Y, bl, Icur, Q, NULL);
}
