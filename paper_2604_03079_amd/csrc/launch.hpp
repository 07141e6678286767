// Host launchers of the HIP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "kernel_args.hpp"

namespace cs {

// Resident blocks per CU of the persistent kernel in `mode` (0 phase-evaluate,
// 1 evaluate-ahead, 2 stamp from buffer) at `block` threads; nc_max = largest number
// of code rows of a device (evaluate-ahead keeps that many values per thread in LDS).
hipError_t persistent_capacity(int mode, int block, int nc_max, int *blocks_per_cu);
hipError_t launch_gather_params(int32_t n, const int32_t *perm, const double *W, const double *L,
                                const double *V, double *par, hipStream_t s);
hipError_t launch_colour_phase(const KCirc &kc, const KCall &call, int c, int count,
                               int with_fixed, hipStream_t s);
hipError_t launch_fixed(const KCirc &kc, const KCall &call, hipStream_t s);
hipError_t launch_hub(const KCirc &kc, const KCall &call, hipStream_t s);
// A[idx[i]] = A[idx[i]] + val[i] for i < n (the linear part of entries that devices
// also write); nothing is launched when n == 0.
hipError_t launch_linear_add(int32_t n, const int32_t *idx, const double *val, double *A, hipStream_t s);
// Damped Newton update: d = y - x, rows below n_clamp clamped to [-vstep, vstep],
// x += d; *step_bits = max over rows of |d| as IEEE bits (NaN above every finite),
// which the caller clears first.
// Level-scheduled sparse LU (solve.hip): T[t] = A[src[t]] (0 where src < 0); one
// lower level: rows eliminated and forward-substituted (y); one upper level: rows
// back-substituted, solution written to out at column Q(i).
hipError_t launch_lu_load(int32_t nnzT, const int32_t *src, const double *A, double *T, hipStream_t s);
hipError_t launch_lu_lower(int32_t count, const int32_t *rows, const int32_t *Tp, const int32_t *Ti,
                           const int32_t *diag, double *T, const int32_t *P, const double *b, double *y,
                           hipStream_t s);
// Same as launch_lu_lower for rows of at most lu_stage_entries() entries, one wave each.
hipError_t launch_lu_lower_wave(int32_t count, const int32_t *rows, const int32_t *Tp, const int32_t *Ti,
                                const int32_t *diag, double *T, const int32_t *P, const double *b, double *y,
                                hipStream_t s);
int32_t lu_stage_entries();
// Caps of k_lu_lower_seq per row: entries, entries left of the diagonal, staged U
// entries (those whose column is in the row).
void lu_seq_caps(int32_t *row, int32_t *l, int32_t *u);
// grid workgroups of one wave, each taking programmed rows in order (prow: 8 ints per
// row): workgroup b rows [b count, (b + 1) count), or [woff[b], woff[b + 1]) when woff
// (device, grid + 1) is given.  One level is grid = its rows and count = 1; a run of
// narrow levels one workgroup per connected part.  Same bits as launch_lu_lower.
hipError_t launch_lu_lower_seq(int32_t grid, int32_t count, const int32_t *woff, const int32_t *prow,
                               const int32_t *plo, const int32_t *pst, double *T, const double *b, double *y,
                               hipStream_t s);
hipError_t launch_lu_upper(int32_t count, const int32_t *rows, const int32_t *Tp, const int32_t *Ti,
                           const int32_t *diag, const double *T, double *y, const int32_t *Q, double *out,
                           hipStream_t s);
// A run of upper levels in one workgroup (lev: nlev + 1 offsets into rows); rows
// with at most 256 entries right of the diagonal; same bits as launch_lu_upper.
hipError_t launch_lu_upper_seq(int32_t nlev, const int32_t *lev, const int32_t *rows, const int32_t *Tp,
                               const int32_t *Ti, const int32_t *diag, const double *T, double *y, const int32_t *Q,
                               double *out, hipStream_t s);
int32_t lu_upper_seq_rows();   // widest level a run takes
hipError_t launch_newton_update(int32_t n, int32_t n_clamp, const uint8_t *clamp, const double *y, double *x,
                                double vstep,
                                unsigned long long *step_bits, hipStream_t s);
// cooperative: hipLaunchCooperativeKernel (the runtime checks co-residency);
// otherwise an ordinary launch of a grid the occupancy query says fits at once.
// n_part: blocks [0, n_part) run the grid-barrier colour schedule over the first
// n_global_chunks hub chunks; later blocks stamp the workgroup-local circuits of kl.
hipError_t launch_persistent(const KCirc &kc, const KCall &call, const KSync &ks,
                             const double *buf, int mode, int grid, int block, bool cooperative,
                             hipStream_t s, int n_part, int n_global_chunks, const KLocal &kl);
// hist_out[4 v + t] = ag0 * Q_t of device v at call.x (call.hist unused).
hipError_t launch_history(const KCirc &kc, const KCall &call, double *hist_out, hipStream_t s);
hipError_t launch_eval_buffer(const KCirc &kc, const KCall &call, double *buf, hipStream_t s);
hipError_t launch_vjp(const KCirc &kc, const KCall &call, const double *A_bar, const double *b_bar,
                      double *gW, double *gL, double *gV, hipStream_t s);
// Region schedule: one workgroup of `block` threads per region; dynamic LDS for
// lds_int interior accumulators plus nc_max merged values per lane (reused as the
// fold scratch).
size_t region_lds_bytes(int lds_int, int nc_max, int block);
hipError_t region_capacity(int block, int lds_int, int nc_max, int *blocks_per_cu);
hipError_t launch_region(const KCirc &kc, const KCall &call, const KRegion &kr, int block, hipStream_t s);
// Grid-barrier form of the region schedule: every region resident at once.
hipError_t region_grid_capacity(int block, int lds_int, int nc_max, int *blocks_per_cu);
hipError_t launch_region_grid(const KCirc &kc, const KCall &call, const KRegion &kr, const KSync &ks, int block,
                              bool cooperative, hipStream_t s);
// dst[j][p] = src[j][idx[p]] for rows j < rows (src rows n_src long, dst rows n).
hipError_t launch_permute_rows(int32_t n, const int32_t *idx, const double *src, int32_t n_src, int32_t rows,
                               double *dst, hipStream_t s);
// Per-device model constants sdp[NSD][kc.n] from kc.par (W, L, VTH0), kc.pol and kc.card.
hipError_t launch_dev_const(const KCirc &kc, double *sdp, hipStream_t s);
hipError_t launch_serial(const KCirc &kc, const KCall &call, int64_t nnz, int64_t n_rows, double *buf,
                         const int32_t *ipos, hipStream_t s);
hipError_t launch_atomic(const KCirc &kc, const KCall &call, int64_t nnz, int64_t n_rows,
                         hipStream_t s);
// The atomic variant with each wave's hub-entry contributions summed before its atomic.
hipError_t launch_atomic_wave(const KCirc &kc, const KCall &call, int64_t nnz, int64_t n_rows, hipStream_t s);

}  // namespace cs
