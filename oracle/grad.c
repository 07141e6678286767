/* Oracle gradient: vector-Jacobian product of the stamped (A, b) with respect to
 * each device's W, L and VTH0.
 *
 * A and b are sums of per-device contributions and each contribution depends on
 * its own device's parameters only, so
 *   dJ/dtheta_k = sum_{(t,u)} Abar[slot(t,u)] * dY_k[t][u]/dtheta_k
 *               + sum_t     bbar[row(t)]    * dbl_k[t]/dtheta_k
 * over the device's non-ground terminals.  The local derivatives are taken by
 * complex-step differentiation of model M at theta_k + i*h, h = 1e-20*|theta_k|.
 */
#include <complex.h>
#include <math.h>

#include "oracle.h"
#include "oracle_internal.h"

void or_device_dparam(const or_card *card, int pol, double W, double L, double VTH0,
                      const double V[4], double ag0, const double *hist, int which,
                      double dY[16], double dbl[4]) {
    or_device_dparam_h(card, pol, W, L, VTH0, V, ag0, hist, which, 1e-20, dY, dbl);
}

void or_device_dparam_h(const or_card *card, int pol, double W, double L, double VTH0,
                        const double V[4], double ag0, const double *hist, int which, double rel_h,
                        double dY[16], double dbl[4]) {
    double th = which == 0 ? W : (which == 1 ? L : VTH0);
    double h = rel_h * fabs(th);
    if (h == 0.0) h = 1e-30;
    double complex Wc = W, Lc = L, Vc = VTH0;
    if (which == 0) Wc = W + I * h;
    else if (which == 1) Lc = L + I * h;
    else Vc = VTH0 + I * h;
    double complex Y[16], bl[4], Ic[4], Q[4];
    or_device_eval_c(card, pol, Wc, Lc, Vc, V, ag0, hist, Y, bl, Ic, Q);
    for (int j = 0; j < 16; ++j) dY[j] = cimag(Y[j]) / h;
    for (int j = 0; j < 4; ++j) dbl[j] = cimag(bl[j]) / h;
}

/* mode 0: the gradient; 1: sum of |cotangent * sensitivity| over the device's
 * stamped entries; 2: the largest |cotangent| of the device times the sum of |d/dtheta|
 * over all 16 local entries and 4 local RHS values (ground terminals included). */
static int vjp_impl(int32_t n_dev, const int32_t *term, const int8_t *pol,
                    const or_card *nmos, const or_card *pmos, const double *W, const double *L,
                    const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
                    const double *x, double ag0, const double *hist, const double *A_bar,
                    const double *b_bar, double *W_bar, double *L_bar, double *VTH0_bar,
                    int mode) {
    for (int32_t v = 0; v < n_dev; ++v) {
        const int32_t *t4 = term + 4 * (int64_t)v;
        double V[4];
        for (int t = 0; t < 4; ++t) V[t] = t4[t] == 0 ? 0.0 : x[t4[t] - 1];
        double *out[3] = {W_bar + v, L_bar + v, VTH0_bar + v};
        for (int which = 0; which < 3; ++which) {
            double dY[16], dbl[4];
            or_device_dparam(pol[v] > 0 ? nmos : pmos, pol[v], W[v], L[v], VTH0[v], V, ag0,
                             hist ? hist + 4 * (int64_t)v : NULL, which, dY, dbl);
            double g = 0.0, cmax = 0.0;
            for (int t = 0; t < 4; ++t) {
                if (t4[t] == 0) continue;
                for (int s = 0; s < 4; ++s) {
                    if (t4[s] == 0) continue;
                    int64_t sl = or_find_slot(row_ptr, col_idx, t4[t] - 1, t4[s] - 1);
                    if (sl < 0) return -3;
                    const double term_ts = A_bar[sl] * dY[t * 4 + s];
                    g += mode == 0 ? term_ts : fabs(term_ts);
                    if (fabs(A_bar[sl]) > cmax) cmax = fabs(A_bar[sl]);
                }
                const double term_t = b_bar[t4[t] - 1] * dbl[t];
                g += mode == 0 ? term_t : fabs(term_t);
                if (fabs(b_bar[t4[t] - 1]) > cmax) cmax = fabs(b_bar[t4[t] - 1]);
            }
            if (mode == 2) {
                double sum = 0.0;
                for (int j = 0; j < 16; ++j) sum += fabs(dY[j]);
                for (int j = 0; j < 4; ++j) sum += fabs(dbl[j]);
                g = cmax * sum;
            }
            *out[which] = g;
        }
    }
    return 0;
}

int or_vjp(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
           const or_card *nmos, const or_card *pmos, const double *W, const double *L,
           const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
           const double *x, double ag0, const double *hist, const double *A_bar,
           const double *b_bar, double *W_bar, double *L_bar, double *VTH0_bar) {
    (void)n_nodes;
    return vjp_impl(n_dev, term, pol, nmos, pmos, W, L, VTH0, row_ptr, col_idx, x, ag0, hist, A_bar,
                    b_bar, W_bar, L_bar, VTH0_bar, 0);
}

/* Per device, sum of |cotangent * local sensitivity| over its entries: the scale of
 * the rounding in a gradient assembled in another order. */
int or_vjp_magnitude(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                     const or_card *nmos, const or_card *pmos, const double *W, const double *L,
                     const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *x, double ag0, const double *hist, const double *A_bar,
                     const double *b_bar, double *W_mag, double *L_mag, double *VTH0_mag) {
    (void)n_nodes;
    return vjp_impl(n_dev, term, pol, nmos, pmos, W, L, VTH0, row_ptr, col_idx, x, ag0, hist, A_bar,
                    b_bar, W_mag, L_mag, VTH0_mag, 1);
}

/* Per device, the largest |cotangent| over its stamped entries and rows times the
 * sum of |d/dtheta| over all its local outputs: the scale of the numbers its
 * sensitivities are formed from.  Entries of the source row and column are negated
 * sums of the others (conservation), and the RHS adds Y (V - V_s) to the currents
 * and charges, so where those cancel (a sensitivity at rounding level beside large
 * ones, e.g. beside an unstamped ground-terminal entry) the oracle's own value is
 * decided by rounding at this scale. */
int or_vjp_round_scale(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                       const or_card *nmos, const or_card *pmos, const double *W, const double *L,
                       const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *x, double ag0, const double *hist, const double *A_bar,
                       const double *b_bar, double *W_s, double *L_s, double *VTH0_s) {
    (void)n_nodes;
    return vjp_impl(n_dev, term, pol, nmos, pmos, W, L, VTH0, row_ptr, col_idx, x, ag0, hist, A_bar,
                    b_bar, W_s, L_s, VTH0_s, 2);
}
