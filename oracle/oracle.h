/* Oracle: plain, serial, FP64 CPU implementation of the coloured MOSFET
 * evaluate-and-stamp step.  TEST INFRASTRUCTURE ONLY: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code with
 * the GPU library.
 *
 * What it computes (paper, Methodology):
 *   - compute phase: each MOSFET instance evaluates its model at the bias point and
 *     yields equivalent conductances and current/charge terms;
 *   - stamp phase: the per-instance contributions are accumulated into the global
 *     sparse MNA matrix A and right-hand side b;
 *   - conflict graph: one vertex per FET, an edge when two FETs share a non-ground
 *     node; greedy colouring (Introduction: smallest colour not used by already
 *     coloured neighbours); colours processed in sequence.
 * The device model is the project's BSIM4-core subset ("model M"): the paper names
 * BSIM 4.82 (Methodology, experimental setup) but prints no equations.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

typedef struct {
    double tnom, toxe, ndep, phis, vbi, k1, k2, k3, w0, dvt0, dvt1, dsub, eta0, nfactor,
        cdsc, voff, u0, ua, ub, uc, vsat, a0, xj, delta, delta1, lambda_l, cgdo, lint, wint;
    /* source/drain-body junctions (jmod = 1): saturation current density js (A/m^2),
     * emission coefficient nj, zero-bias capacitance cj (F/m^2) of an abrupt
     * junction (grading 1/2), built-in potential pb (V), forward-bias coefficient
     * fc, diffusion length hdif (junction area = Weff * hdif), forward voltage vjmax
     * (V, at most 40 nj VT) above which the diode is continued by its tangent */
    double jmod, js, nj, cj, pb, fc, hdif, vjmax;
} or_card;

/* Intermediate values of one evaluation (value parts), for the model checks. */
typedef struct {
    int mode;
    double x1, x2, x3;
    double theta_sce, theta_dibl, vth_s, beta0, lambda, abl, cg, cov;
    double vbseff, sqps, vth, n, vgst, vgsteff, mu, esatl, abulk, v2, vdsat, vdseff, ids0, ids;
    double vdc, vdcv, qinv, qb, qd, qs, qg;
    double dids[3];  /* dIds / d(x1, x2, x3) in the evaluation frame */
} or_trace;

/* Elementary functions (project definitions, see elem.c). */
double or_pexp(double a);
double or_plog1p(double y);
double or_softplus(double t);
double or_sigma(double t);
double or_pcosh(double u);
void or_elem_array(int kind, const double *x, double *y, int64_t n);

/* FP64 operation counter for model M (+, -, *, /, sqrt each count 1). */
void or_count_ops(int on);
long long or_ops(void);
/* Operations of the size-dependent constants (W, L, VTH0 only) in the last counted
 * device evaluation: work done once per parameter set, not per Newton iteration. */
long long or_sizedep_ops(void);

/* One device: V = terminal voltages (d, g, s, b).  Outputs Y[4][4] row-major
 * (rows/cols d, g, s, b), bl[4], physical terminal currents I[4] and charges Q[4].
 * hist may be NULL. tr may be NULL. */
void or_device_eval(const or_card *card, int pol, double W, double L, double VTH0,
                    const double V[4], double ag0, const double *hist, double Y[16],
                    double bl[4], double Icur[4], double Q[4], or_trace *tr);

/* Greedy colouring in ascending device order.  excl: n_nodes flags (NULL = only
 * ground is non-conflicting).  Returns 0 on success. */
int or_colour(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl,
              int32_t *colour, int32_t *n_colours, int64_t *n_edges);

/* Colouring in another vertex order: 0 ascending index (or_colour), 1 largest
 * degree first, 2 DSATUR.  Same conventions as or_colour; quadratic time. */
int or_colour_order(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl, int order,
                    int32_t *colour, int32_t *n_colours, int64_t *n_edges);

/* CSR pattern.  res: 2*n_res node pairs of series resistors (may be NULL when
 * n_res == 0).  row_ptr has n_rows+1 entries; col_idx must hold at least
 * 16*n_dev + n_rows + 4*n_vsrc + 2*n_res entries.  *nnz receives the count. */
int or_pattern(int32_t n_nodes, int32_t n_dev, const int32_t *term, int32_t n_vsrc,
               const int32_t *vsrc, int32_t n_res, const int32_t *res, int32_t *row_ptr,
               int32_t *col_idx, int64_t *nnz);

/* Linear part of the matrix: resistor j (conductance g[j], nodes res[2j], res[2j+1])
 * stamps +g, -g, -g, +g at (p,p), (p,q), (q,p), (q,q), ground dropped.  Lin (nnz
 * values) starts at zero and takes the stamps in resistor order; touched flags the
 * entries that received any.  magnitude: |stamp|.  -2 bad node, -3 entry missing. */
int or_linear_stamp(int32_t n_nodes, int32_t n_res, const int32_t *res, const double *g,
                    const int32_t *row_ptr, const int32_t *col_idx, int64_t nnz, double *Lin,
                    uint8_t *touched, int magnitude);

/* Expected stamp map in original device order: slot[16*v + j] (j < k*k, else -1),
 * sflag (0 add, 1 store, 2 hub), brow[4*v + a] (a < k, else -1), bflag. */
int or_stamp_map(int32_t n_nodes, int32_t n_dev, const int32_t *term, const uint8_t *excl,
                 const int32_t *colour, const int32_t *row_ptr, const int32_t *col_idx,
                 int32_t *slot, int8_t *sflag, int32_t *brow, int8_t *bflag);

/* Assembly of A (CSR values) and b.  colour == NULL: serial order (devices
 * ascending, A and b zero-initialised, +=).  Otherwise colour replay (colours
 * ascending; first writer stores, later writers add; hub outputs summed by
 * or_hubsum in ascending device order).  excl (replay only) defines hub outputs.
 * Then, in both orders, each entry touched by a series resistor gets its linear
 * part (or_linear_stamp) added once. */
int or_assemble(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                int32_t n_vsrc, const int32_t *vsrc, const double *vsrc_volts,
                int32_t n_res, const int32_t *res, const double *res_g, const or_card *nmos,
                const or_card *pmos, const double *W, const double *L, const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
                const int32_t *colour, const uint8_t *excl, const double *x, double ag0,
                const double *hist, double *A, double *b);

/* Colour replay (colour != NULL required) with the compute phase and each colour's
 * devices spread over the OpenMP threads: the same bits as or_assemble's colour
 * replay.  or_omp_threads: the number of threads it uses. */
int or_assemble_omp(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                    int32_t n_vsrc, const int32_t *vsrc, const double *vsrc_volts,
                    int32_t n_res, const int32_t *res, const double *res_g, const or_card *nmos,
                    const or_card *pmos, const double *W, const double *L, const double *VTH0,
                    const int32_t *row_ptr, const int32_t *col_idx, const int32_t *colour,
                    const uint8_t *excl, const double *x, double ag0, const double *hist, double *A,
                    double *b);
int or_omp_threads(void);

/* Per entry, the sum of |contribution| over devices (serial order): the scale of
 * the rounding difference between two accumulation orders. */
int or_assemble_magnitude(int32_t n_nodes, int32_t n_dev, const int32_t *term,
                          const int8_t *pol, int32_t n_vsrc, const int32_t *vsrc,
                          const double *vsrc_volts, int32_t n_res, const int32_t *res,
                          const double *res_g, const or_card *nmos, const or_card *pmos,
                          const double *W, const double *L, const double *VTH0,
                          const int32_t *row_ptr, const int32_t *col_idx, const double *x,
                          double ag0, const double *hist, double *A, double *b);

/* Fixed-shape hub sum: the pairwise tree sum, split at the largest power of two
 * below m (a perfect binary tree over the contributions padded with -0.0). */
double or_hubsum(const double *c, int64_t m);

/* Vector-Jacobian product of (A, b) with respect to per-device W, L, VTH0 by
 * complex-step differentiation of each device's local outputs. */
int or_vjp(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
           const or_card *nmos, const or_card *pmos, const double *W, const double *L,
           const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
           const double *x, double ag0, const double *hist, const double *A_bar,
           const double *b_bar, double *W_bar, double *L_bar, double *VTH0_bar);

/* Per device, sum over its entries of |cotangent * d(entry)/d(theta)|. */
int or_vjp_magnitude(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                     const or_card *nmos, const or_card *pmos, const double *W, const double *L,
                     const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
                     const double *x, double ag0, const double *hist, const double *A_bar,
                     const double *b_bar, double *W_mag, double *L_mag, double *VTH0_mag);

/* Per device, max |cotangent| over its stamped entries and rows times the sum of
 * |d(local output)/d(theta)| over all 16 local entries and 4 RHS values: the rounding
 * scale of its sensitivities where conservation sums cancel. */
int or_vjp_round_scale(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                       const or_card *nmos, const or_card *pmos, const double *W, const double *L,
                       const double *VTH0, const int32_t *row_ptr, const int32_t *col_idx,
                       const double *x, double ag0, const double *hist, const double *A_bar,
                       const double *b_bar, double *W_s, double *L_s, double *VTH0_s);

/* Per-device local sensitivities d(Y, bl)/d(theta) by complex step, theta = 0 (W),
 * 1 (L), 2 (VTH0).  dY[16], dbl[4].  The step is i * 1e-20 * |theta|; the _h form
 * takes the relative step (two steps give two exact derivatives of the same rounded
 * program, which differ only where that derivative is ill-conditioned). */
void or_device_dparam(const or_card *card, int pol, double W, double L, double VTH0,
                      const double V[4], double ag0, const double *hist, int which,
                      double dY[16], double dbl[4]);
void or_device_dparam_h(const or_card *card, int pol, double W, double L, double VTH0,
                        const double V[4], double ag0, const double *hist, int which, double rel_h,
                        double dY[16], double dbl[4]);

#endif
