/* Oracle internals shared between the oracle's own translation units. */
#ifndef ORACLE_INTERNAL_H
#define ORACLE_INTERNAL_H
#include <complex.h>
#include <stddef.h>
#include <stdint.h>

#include "oracle.h"

extern long long or_opcount_;
extern long long or_sizedep_ops_;
extern int or_counting_;
#define OR_COUNT(n) do { if (or_counting_) or_opcount_ += (n); } while (0)

double complex or_cpexp(double complex a);
double complex or_cplog1p(double complex y);
double complex or_csoftplus(double complex t);
double complex or_csigma(double complex t);
double complex or_cpcosh(double complex u);

/* Complex-parameter evaluation (complex-step); same equations as or_device_eval. */
void or_device_eval_c(const or_card *card, int pol, double complex W, double complex L,
                      double complex VTH0, const double V[4], double ag0, const double *hist,
                      double complex Y[16], double complex bl[4], double complex Icur[4],
                      double complex Q[4]);

/* Unique non-ground nodes of a device in first-appearance order over (d, g, s, b).
 * Returns k; a[t] = index of terminal t's node in u[], or -1 for ground. */
int or_unique_nodes(const int32_t term4[4], int32_t u[4], int a[4]);

/* Position of column c in CSR row r, or -1. */
int64_t or_find_slot(const int32_t *row_ptr, const int32_t *col_idx, int32_t r, int32_t c);

#endif
