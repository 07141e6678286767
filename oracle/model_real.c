/* Real (binary64) instantiation of model M: the values the GPU must reproduce
 * bit for bit. */
#include <math.h>

#include "oracle.h"
#include "oracle_internal.h"

#define T double
#define FN(name) name##_r
#define S_SQRT sqrt
#define S_PEXP or_pexp
#define S_SOFTPLUS or_softplus
#define S_SIGMA or_sigma
#define S_PCOSH or_pcosh
#define S_PLOG1P or_plog1p
#define S_RE(x) (x)
#define CNT(n) OR_COUNT(n)
#define SIZEDEP_BEGIN const long long sizedep0_ = or_opcount_
#define SIZEDEP_END or_sizedep_ops_ = or_opcount_ - sizedep0_
#define WITH_TRACE 1
#include "model_m.inc"

void or_device_eval(const or_card *card, int pol, double W, double L, double VTH0,
                    const double V[4], double ag0, const double *hist, double Y[16],
                    double bl[4], double Icur[4], double Q[4], or_trace *tr) {
    or_device_eval_r(card, pol, W, L, VTH0, V, ag0, hist, Y, bl, Icur, Q, tr);
}
