/* colorstamp: coloured, conflict-free MOSFET evaluate-and-stamp on MI355X (gfx950).
 *
 * The operation (paper "EEspice: A Modular Circuit Simulation Platform with Parallel
 * Device Model Evaluation via Graph Coloring"):
 *   - Introduction / Methodology: each Newton-Raphson iteration evaluates every
 *     device model at the present operating point (compute phase: equivalent
 *     conductances and current/charge terms) and stamps the contributions into the
 *     shared MNA matrix A and right-hand side b (stamp phase);
 *   - Methodology: the FET conflict graph (one vertex per FET, an edge when two FETs
 *     share a non-ground node) is built at circuit setup and coloured greedily; the
 *     NR loop processes colours sequentially and evaluates and stamps all devices of
 *     a colour in parallel, without locks;
 *   - Table "Summary of BSIM4 evaluation-kernel variants": kernels are
 *     interchangeable without changing the simulation loop (cs_variant below).
 *
 * Conventions
 *   - Nodes: 0 is ground.  MNA rows: non-ground node n -> row n-1, then one branch row
 *     per voltage source, in source order.  A is CSR with sorted, unique columns:
 *     every ordered pair of a device's non-ground terminal nodes, every node-row
 *     diagonal, and (pos, br), (br, pos) (and neg likewise) per voltage source.
 *   - Device terminals are (d, g, s, b); pol = +1 NMOS, -1 PMOS.
 *   - Ownership: create copies every host input; the library owns its setup buffers
 *     (host and device).  x, A, b, W, L, VTH0, hist, cotangents and gradients are
 *     caller-owned DEVICE memory (FP64).  Streams are hipStream_t passed as void*.
 *   - Calls are stream-ordered and asynchronous.  Argument and state errors are
 *     detected on the host before any launch; a failed launch returns CS_EHIP.
 *     No exceptions cross the ABI.  cs_last_error() describes the last failure of
 *     the calling thread.  A handle is used by one stream at a time.
 *   - cs_eval_stamp overwrites every entry of A_val and b (no zero-fill contract).
 */
#ifndef COLORSTAMP_H
#define COLORSTAMP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cs_circuit cs_circuit;
typedef struct cs_batch cs_batch;

typedef enum {
    CS_OK = 0,
    CS_EINVAL = -1,   /* bad argument: null pointer, node id, polarity or size */
    CS_ENOMEM = -2,   /* host or device allocation failed */
    CS_EHIP = -3,     /* a HIP runtime call or kernel launch failed */
    CS_ESTATE = -4,   /* calls out of order (e.g. evaluate before the stamp map) */
    CS_ENOTSUP = -5,  /* size or configuration beyond what the library supports */
    CS_EDOMAIN = -6   /* a kernel reported a failed bounded wait (see cs_check) */
} cs_status;

/* Kernel variants (paper, Table "Summary of BSIM4 evaluation-kernel variants"). */
typedef enum {
    CS_COLOR_PERSISTENT = 0,  /* ColorFused: one persistent kernel; colours in sequence,
                                 grid-wide barrier between colours; plain stores and
                                 load-adds only.  When every region of the region
                                 schedule fits on the GPU at once, the same launch runs
                                 that schedule with a grid-wide barrier between levels
                                 of shared entries instead (same bits). */
    CS_COLOR_PER_KERNEL = 1,  /* ColorFused with one kernel launch per colour (the
                                 per-colour parallel-for of the paper's OpenMP form) */
    CS_ATOMIC = 2,            /* comparison: no colouring, FP64 atomic adds (the
                                 paper's lock-based foil, Introduction) */
    CS_COLOR_BUFFERED = 3,    /* Color: evaluate every device into a buffer, then
                                 stamp colour by colour from the buffer */
    CS_COLOR_REGION = 4,      /* ColorFused at workgroup scope: devices are cut (in
                                 index order) into regions of one workgroup; an entry
                                 written by one or two devices of a region accumulates
                                 in LDS by LDS atomic adds (exact for two writers),
                                 one written by more devices of a
                                 region is folded by one lane in colour order, and
                                 entries written from several regions are staged and
                                 folded in colour order by the last contributing
                                 region.  Same bits as CS_COLOR_PERSISTENT; no
                                 grid-wide barrier. */
    CS_SERIAL_STAMP = 5,      /* loadomp: evaluate every device into a buffer in
                                 parallel, then one lane adds every device's values in
                                 ascending device index onto zeroed A and b (the serial
                                 order of accumulation, hub entries included). */
    CS_ATOMIC_WAVE = 6        /* comparison: CS_ATOMIC with each wave's contributions to
                                 a hub (rail) entry summed over the wave first and added
                                 with one atomic, so that the comparison measures
                                 lock-free stamping rather than contention on the
                                 rails (without excluded rails it equals CS_ATOMIC) */
} cs_variant;

/* Model card of the BSIM4-core subset (SI units).  One card per polarity.  The
 * last fields select the second model level: jmod = 1 adds the source- and drain-
 * body junctions of BSIM4 (diode current Is (e^(v/(nj VT)) - 1), Is = js Weff hdif,
 * exponent clamped at -40 and continued by its tangent above vjmax <= 40 nj VT;
 * abrupt-junction depletion charge, cj Weff hdif at zero bias, continued with a
 * linear capacitance above fc pb); jmod = 0 is model M exactly.  CS_EINVAL from
 * cs_set_models for jmod = 1 with nj <= 0, pb <= 0, fc outside [0, 1), negative
 * js, cj or hdif, or vjmax above 40 nj VT. */
typedef struct {
    uint32_t size;  /* = sizeof(cs_model_card) */
    double tnom, toxe, ndep, phis, vbi, k1, k2, k3, w0, dvt0, dvt1, dsub, eta0, nfactor,
        cdsc, voff, u0, ua, ub, uc, vsat, a0, xj, delta, delta1, lambda_l, cgdo, lint, wint;
    double jmod, js, nj, cj, pb, fc, hdif, vjmax;
} cs_model_card;

/* Create a circuit.  term: n_dev*4 node ids (d, g, s, b), 0 <= id < n_nodes;
 * pol: n_dev entries of +1/-1; vsrc: n_vsrc*2 (pos, neg) node ids; vsrc_volts:
 * n_vsrc values.  All host pointers, copied.  *out receives the handle. */
cs_status cs_circuit_create(int32_t n_nodes, int32_t n_dev, const int32_t *term,
                            const int8_t *pol, int32_t n_vsrc, const int32_t *vsrc,
                            const double *vsrc_volts, cs_circuit **out);
void cs_circuit_destroy(cs_circuit *c);

/* Series resistors of a split netlist (Benchmark 2: Table I's R14 and R89 adders,
 * where small resistors cut shared nets so fewer FETs conflict).  nodes: n_res*2
 * (p, q) node ids, 0 <= id < n_nodes (0 ground); g: n_res conductances in siemens,
 * finite.  Host pointers, copied; a later call replaces the set (n_res = 0 clears).
 * Resistors are linear and do not enter the FET conflict graph: each adds +g at
 * (p,p) and (q,q) and -g at (p,q) and (q,p) of A (ground rows and columns
 * dropped), nothing to b.  Per entry these stamps are summed from zero in resistor
 * order, and the sum is added once to A after every device contribution (an entry
 * no device writes receives 0 + sum).  Must precede cs_build_stamp_map (CS_ESTATE
 * after it, until the next colouring). */
cs_status cs_set_resistors(cs_circuit *c, int32_t n_res, const int32_t *nodes, const double *g);

/* Conflict graph and greedy colouring (Methodology; Introduction for the greedy
 * rule).  exclude: n_nodes host flags of nodes that do not create conflicts (NULL:
 * only ground, the paper's rule).  Devices are visited in ascending index and take
 * the smallest colour unused by an already coloured neighbour.  Entries whose row
 * and column nodes are both excluded (and b rows of excluded nodes) become hub
 * entries, summed by a fixed-shape reduction.  Outputs (each may be NULL): number
 * of colours, colour per device (host, n_dev), number of conflict edges. */
cs_status cs_build_coloring(cs_circuit *c, const uint8_t *exclude, int32_t *n_colors,
                            int32_t *colour_out, int64_t *n_edges);

/* Vertex orders of the greedy colouring. */
typedef enum {
    CS_ORDER_NATURAL = 0,        /* ascending device index (the paper's; cs_build_coloring) */
    CS_ORDER_LARGEST_FIRST = 1,  /* decreasing conflict degree, ties by ascending index
                                    (Welsh and Powell) */
    CS_ORDER_DSATUR = 2          /* most distinct colours among coloured neighbours first,
                                    ties by larger degree, then smaller index (Brelaz) */
} cs_colour_order;

/* cs_build_coloring with another vertex order (same outputs and conventions; every
 * later step works with any proper colouring).  CS_EINVAL for an unknown order. */
cs_status cs_build_coloring_order(cs_circuit *c, const uint8_t *exclude, int32_t order, int32_t *n_colors,
                                  int32_t *colour_out, int64_t *n_edges);

/* CSR pattern and the device-to-slot stamp map (Methodology: stamps touch common
 * MNA rows/columns).  The pattern holds every node pair of a device, every node
 * diagonal, the voltage-source pairs and each resistor's (p,q), (q,p).  Requires
 * cs_build_coloring.  Uploads topology and map to the current HIP device.
 * Outputs: number of rows and nonzeros. */
cs_status cs_build_stamp_map(cs_circuit *c, int32_t *n_rows, int64_t *nnz);

/* Host copies of the pattern: row_ptr[n_rows+1], col_idx[nnz]. */
cs_status cs_get_pattern(const cs_circuit *c, int32_t *row_ptr, int32_t *col_idx);

/* Host copy of the stamp map in original device order: slot[16*v + j] for
 * j < k*k (k = distinct non-ground nodes of device v, in first-appearance order over
 * d, g, s, b; entry j = a*k + b is node pair (a, b)), -1 beyond; sflag: 0 load-add,
 * 1 plain store (first writer in colour order), 2 hub; brow[4*v + a] = row of node a,
 * -1 beyond; bflag likewise.  Any pointer may be NULL. */
cs_status cs_get_stamp_map(const cs_circuit *c, int32_t *slot, int8_t *sflag, int32_t *brow,
                           int8_t *bflag);

/* Model cards (host pointers, copied; size field checked). */
cs_status cs_set_models(cs_circuit *c, const cs_model_card *nmos, const cs_model_card *pmos);

/* Per-device parameters in original device order (device pointers, n_dev each).
 * Copied into the library's colour-major layout (and, when the region schedule's
 * tables are on the device, its region-major copy) by kernels on `stream`, so a
 * captured evaluate-and-stamp replayed after this call reads the new values.  The
 * library's copies keep their addresses until the next colouring or stamp map. */
cs_status cs_set_params(cs_circuit *c, const double *W, const double *L, const double *VTH0,
                        void *stream);

/* Evaluate every device at x (device, n_rows) and stamp A_val (device, nnz) and b
 * (device, n_rows).  ag0: charge-to-current coefficient of the integration formula
 * (0 for a DC stamp); hist: device, n_dev*4 history terms in original device order,
 * or NULL.  Per device the local conductance matrix Y = dI/dV + ag0*dQ/dV and
 * right-hand side Y*(V - Vs) - I - ag0*Q (+ hist) are merged onto its node pairs and
 * accumulated: colour by colour, first writer stores, later writers add.  The
 * linear part of the series resistors (cs_set_resistors) follows on `stream`. */
cs_status cs_eval_stamp(cs_circuit *c, cs_variant variant, const double *x, double ag0,
                        const double *hist, double *A_val, double *b, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): cs_eval_stamp with the
 * region schedule (CS_COLOR_REGION, same bits), calling no hipMalloc, hipFree or
 * other allocating routine.  Its scratch memory (the staging array of shared-entry
 * and hub contributions, the hub chunk sums and the arrival counters) lives in one
 * library-wide device array of CS_NOALLOC_SCRATCH_BYTES per GPU, held until the
 * process ends, instead of the circuit's own buffers; its counters are cleared by a
 * kernel at the start of every call.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other threads) race, so the caller
 * orders them.  Requires the region tables on the device for the circuit's current
 * block size, which one cs_eval_stamp with CS_COLOR_REGION uploads (CS_ESTATE
 * otherwise).  CS_ENOTSUP when the circuit's scratch exceeds the array (the
 * message gives both sizes).  Arguments, ownership and other errors as in
 * cs_eval_stamp. */
#define CS_NOALLOC_SCRATCH_BYTES (16u << 20)
cs_status cs_eval_stamp_noalloc(cs_circuit *c, const double *x, double ag0, const double *hist, double *A_val,
                                double *b, void *stream);

/* Newton-Raphson loop around cs_eval_stamp (Introduction: each iteration evaluates
 * the devices at x, stamps the linearised MNA system and solves it; the paper solves
 * with KLU, Benchmark 2).  Per iteration on `stream`: cs_eval_stamp(variant) into
 * A_val and b (caller-owned device workspace, nnz and n_rows), a sparse LU
 * refactorisation of A and its triangular solves by `solver` (cs_solver), with the
 * pivots of one host factorisation made at the first call on this stamp map
 * (voltage sources first as node/branch pivot pairs, then nested dissection;
 * threshold partial pivoting), leaving the Newton point y in b, then
 * d = y - x with node rows clamped to [-vstep, vstep], x += d.  Stops when
 * max |d| <= tol or after max_iter iterations.  x: device, n_rows, the start point
 * on entry and the last iterate on return.  ag0 and hist as in cs_eval_stamp (a
 * backward-Euler step when ag0 > 0; ag0 = 0 is a DC operating point).  Host
 * outputs (each may be NULL): iterations done, converged (0/1), max |d| of the
 * last iteration, times_ms[5] = summed milliseconds of stamping, refactorisation,
 * solve and update, and the one-time host factorisation.  Returns CS_OK whether or
 * not it converged; CS_EDOMAIN when a step is not finite (x then holds it) or the
 * host factorisation finds the matrix singular. */
typedef enum {
    CS_SOLVE_LEVELS = 0,     /* this library's kernels: rows of the factor pattern grouped by
                                dependency level, one launch per level (refactorisation fused
                                with the forward substitution, then the backward one) */
    CS_SOLVE_ROCSOLVER = 1   /* rocSOLVER csrrf refactorisation and solve, same pivots */
} cs_solver;

cs_status cs_newton(cs_circuit *c, cs_variant variant, int32_t solver, double *x, double ag0,
                    const double *hist, int32_t max_iter, double vstep, double tol, double *A_val,
                    double *b, int32_t *n_iter, int32_t *converged, double *last_step,
                    double *times_ms, void *stream);

/* Schedule options of cs_newton's level-scheduled solver (bits; 0 = default, all
 * on).  CS_NEWTON_NO_PROGRAMMED_ROWS: every lower row by the per-level staged or
 * per-lane kernels (no host program, no runs of narrow levels).
 * CS_NEWTON_NO_UPPER_RUNS: every upper level in its own launch.  The options change
 * launches only: the iterates are the same bits.  The next cs_newton plans again
 * (its host factorisation included).  CS_EINVAL for an unknown bit. */
enum {
    CS_NEWTON_NO_PROGRAMMED_ROWS = 1,
    CS_NEWTON_NO_UPPER_RUNS = 2
};
cs_status cs_set_newton_options(cs_circuit *c, int32_t flags);

/* History terms of the next backward-Euler step (the integration the hist argument
 * of cs_eval_stamp and cs_newton serves: the charge current is ag0 (Q(x) - Q(x_prev))
 * with ag0 = 1/h).  hist_out (device, n_dev*4, original device order, terminals d, g,
 * s, b) receives ag0 * Q_t of every device at x (device, n_rows).  Model M's charges,
 * the same values and operation order as its stamp. */
cs_status cs_history(cs_circuit *c, const double *x, double ag0, double *hist_out, void *stream);

/* The host factorisation cs_newton starts from, for inspection: A_host holds nnz
 * values on the circuit's pattern.  *nnzT receives the size of T = (L - I) + U of
 * P A Q (CSR over the permuted indices, columns ascending); P[k] is the row and Q[k]
 * the column taken at step k.  Arrays (n_rows, n_rows, n_rows+1, nnzT, nnzT) may be
 * NULL; call once with them NULL for the size.  CS_EDOMAIN if singular. */
cs_status cs_factor_host(const cs_circuit *c, const double *A_host, int64_t *nnzT, int32_t *P,
                         int32_t *Q, int32_t *ptrT, int32_t *indT, double *valT);

/* Vector-Jacobian product of the stamped (A, b) with respect to W, L, VTH0:
 * W_bar[k] = sum_j A_bar[slot] * dA_contrib/dW_k + sum_r b_bar[r] * db_contrib/dW_k,
 * likewise L and VTH0.  All pointers are device memory in original device order;
 * model intermediates are recomputed, not stored. */
cs_status cs_vjp(cs_circuit *c, const double *x, double ag0, const double *hist,
                 const double *A_bar, const double *b_bar, double *W_bar, double *L_bar,
                 double *VTH0_bar, void *stream);

/* Launch configuration.  block: threads per block (64, 128, 192 or 256; 0 =
 * default 256); eval_ahead: 1 = the persistent kernel evaluates every device before
 * the colour phases and keeps the results in registers (requires the resident grid
 * to hold one device per thread), 0 = evaluate inside each colour phase, -1 =
 * choose; cooperative: 1 = hipLaunchCooperativeKernel (the runtime guarantees that
 * every block is resident), 0 = an ordinary launch of a grid that the occupancy
 * query says fits the device at once (lower launch cost; the caller must not run
 * other work on the device concurrently - a block that cannot become resident makes
 * the bounded barrier waits expire, reported by cs_check as CS_EDOMAIN). */
cs_status cs_set_launch(cs_circuit *c, int32_t block, int32_t eval_ahead, int32_t cooperative);

/* Sizes and launch facts: n_dev, n_rows, nnz, n_colors, grid (persistent kernel
 * blocks), block, eval_ahead in use, number of hub entries.  Any pointer may be NULL. */
cs_status cs_get_info(const cs_circuit *c, int64_t *n_dev, int32_t *n_rows, int64_t *nnz,
                      int32_t *n_colors, int32_t *grid, int32_t *block, int32_t *eval_ahead,
                      int32_t *n_hub);

/* Region schedule (CS_COLOR_REGION).  The plan is built on the host for a region
 * capacity of `block` threads, by this call or by the first CS_COLOR_REGION call
 * at the current block size (cs_set_launch).  Host only; no device work. */
cs_status cs_plan_regions(cs_circuit *c, int32_t block);

/* Facts of the last region plan: regions (= workgroups), largest number of phases
 * of a region, items (entries shared between regions, and hub chunks), staged
 * contributions (hub and shared), entries owned by one region and accumulated in
 * its LDS (one or two writers), region-to-item links, lane folds (entries owned by
 * one region with three or more writers) and their writer references.
 * Any pointer may be NULL; zeros before a plan exists. */
cs_status cs_get_region_info(const cs_circuit *c, int32_t *n_regions, int32_t *max_phases,
                             int64_t *n_items, int64_t *n_staged, int64_t *n_interior,
                             int64_t *n_links, int64_t *n_folds, int64_t *n_fold_src);

/* Host copies of the region plan tables (any pointer may be NULL), region-major
 * positions p < n_dev:
 *   perm[p]      device index;               phase[p]   phase of the device (an order
 *                                            in which plain LDS loads and stores
 *                                            would accumulate; the kernel adds with
 *                                            LDS atomics instead);
 *   code[j*n_dev + p] (j < 20): bits 31..30 = 0 LDS add, 1 LDS store, 2 staged,
 *                3 unused or read by a lane fold or a local hub chunk; bits 29..0 =
 *                LDS slot or staging index;
 *   rtab[12*r ...] first position, NMOS count, PMOS count (NMOS lanes first, then
 *                PMOS), phases, owned-entry range, item range, lane-fold range,
 *                local hub part range (cs_get_region_hubs);
 *   interior[i]  target of owned entry i (bits 31..30 = 0 A slot, 1 b row), LDS slot =
 *                i - range start;
 *   links[]      item ids per region;
 *   item[4*i ...] first staged index, count, target (kind 0 A, 1 b, 2 hub part),
 *                number of contributing regions (0: an entry with more than 8
 *                contributions, folded by the follow-up kernel of the schedule);
 *   fold[3*i ...] target (as for interior), first index in fold_src, writer count;
 *   fold_src[]   writers of a lane fold in colour order, each (code row j << 16) |
 *                lane of the writer within its region: one lane of the region folds
 *                the writers' merged values left and stores the entry. */
cs_status cs_get_region_plan(const cs_circuit *c, int32_t *perm, uint16_t *phase, int32_t *code,
                             int32_t *rtab, int32_t *interior, int32_t *links, int32_t *item,
                             int32_t *fold, int32_t *fold_src);

/* Hub tables of the region plan (any table pointer may be NULL).  The schedule sums a
 * hub entry (reading of the conflict rule with excluded rails, Methodology) by the
 * pairwise tree over its contributions in ascending device index, in parts: aligned
 * chunks of 32 contributions (subtrees of that tree), then the tree over the parts.
 * A part whose contributions all come from one region is summed by that region: its
 * k-th such part occupies the 32 LDS slots after the region's owned entries and
 * 32 k before (code tag 1, slot r = contribution r of the part; unused slots keep
 * their -0.0 start).  A part spanning regions, or one that would not fit the
 * region's LDS, is an item (kind 2) over its staged contributions.  A follow-up
 * kernel of the schedule sums each hub's parts.  counts[2]: local parts, hubs;
 * hfold[i]: part index of local part i (rtab fields 10, 11 give each region's
 * range); part_ptr[hubs + 1]: part ranges per hub. */
cs_status cs_get_region_hubs(const cs_circuit *c, int64_t *counts, int32_t *hfold, int32_t *part_ptr);

/* Read and clear the device error word of the last bounded waits (synchronises the
 * stream).  Returns CS_EDOMAIN if a barrier wait ran out of its spin budget. */
cs_status cs_check(cs_circuit *c, void *stream);

/* Spin budget of the persistent kernel's barrier waits (iterations; 0 = default). */
cs_status cs_set_spin_limit(cs_circuit *c, int64_t spins);

/* Compute units the region planner sizes the last regions for: -1 (default) = the
 * current GPU's count, 0 = no sizing, n > 0 = n units.  When the full regions
 * (block devices each) fill their last dispatch round on only a few units (at most
 * a quarter), that round is cut into regions of 64 devices, so its extra waves
 * spread over more units.  Takes effect at the next planning. */
cs_status cs_set_plan_units(cs_circuit *c, int32_t cus);

/* ---- batches: many independent circuits stamped in one launch ------------------
 * The batch packs its circuits (each already coloured and mapped, models set) into
 * one instance table.  Packed layouts concatenate per-circuit arrays in batch order:
 * x and b by rows, A by nonzeros, W/L/VTH0 and gradients by devices, hist by 4*devices.
 * Offsets come from cs_batch_layout. */
cs_status cs_batch_create(int32_t n, cs_circuit *const *circuits, cs_batch **out);
void cs_batch_destroy(cs_batch *b);
/* Offsets (host arrays of n+1 entries each; any may be NULL). */
cs_status cs_batch_layout(const cs_batch *b, int64_t *dev_off, int64_t *row_off,
                          int64_t *nnz_off);
/* As cs_set_params, over the packed device order. */
cs_status cs_batch_set_params(cs_batch *b, const double *W, const double *L,
                              const double *VTH0, void *stream);
/* Launch configuration of the batched persistent kernel (see cs_set_launch) and the
 * size up to which a circuit is stamped inside one workgroup with workgroup
 * barriers (colour-phase fusion; 0 = off). */
cs_status cs_batch_set_launch(cs_batch *b, int32_t block, int32_t eval_ahead,
                              int32_t local_max_dev);
cs_status cs_batch_get_info(const cs_batch *b, int64_t *n_dev, int64_t *n_rows, int64_t *nnz,
                            int32_t *max_colors, int32_t *grid, int32_t *block,
                            int32_t *eval_ahead, int32_t *n_local);
/* Schedule of cs_batch_eval_stamp: CS_COLOR_PERSISTENT (default; grid-barrier
 * colour phases for circuits above local_max_dev devices, workgroup-local ones
 * below) or CS_COLOR_REGION (every circuit cut into workgroup regions, small
 * circuits packed whole into regions; see cs_variant). */
cs_status cs_batch_set_schedule(cs_batch *b, cs_variant schedule);
/* Batch analogues of cs_plan_regions, cs_get_region_info and cs_get_region_plan
 * (positions and devices over the packed device order; circuits that fit one
 * region are never split).  Host only. */
cs_status cs_batch_plan_regions(cs_batch *b, int32_t block);
cs_status cs_batch_get_region_info(const cs_batch *b, int32_t *n_regions, int32_t *max_phases,
                                   int64_t *n_items, int64_t *n_staged, int64_t *n_interior,
                                   int64_t *n_links, int64_t *n_folds, int64_t *n_fold_src);
cs_status cs_batch_get_region_plan(const cs_batch *b, int32_t *perm, uint16_t *phase, int32_t *code,
                                   int32_t *rtab, int32_t *interior, int32_t *links, int32_t *item,
                                   int32_t *fold, int32_t *fold_src);
cs_status cs_batch_get_region_hubs(const cs_batch *b, int64_t *counts, int32_t *hfold, int32_t *part_ptr);
/* A launch configuration of cs_batch_eval_stamp (see cs_batch_set_launch and
 * cs_batch_set_schedule) and its measured time. */
typedef struct {
    int32_t schedule;        /* CS_COLOR_PERSISTENT or CS_COLOR_REGION */
    int32_t block;           /* threads per workgroup */
    int32_t eval_ahead;      /* persistent schedule: -1 choose, 0 evaluate in each phase */
    int32_t local_max_dev;   /* persistent schedule: circuits up to this size inside one workgroup */
    double ms;               /* mean time of one batched step, milliseconds */
} cs_batch_config;

/* Autotuner of the batched launch (a sizing loop calls the simulator repeatedly on
 * one batch, Introduction).  Every candidate configuration (persistent schedule:
 * block 128 or 256 x local_max_dev 0, 64, 256, 1024, 4096 x eval_ahead -1, 0;
 * region schedule: block 128, 192, 256) is applied, its parameters gathered from
 * W, L, VTH0 (device, packed device order), one batched step at x (device, packed
 * rows) is captured in a HIP graph on `stream` and replayed `reps` times between two
 * events; A and b_vec (device, packed) are the step's workspace and hold its last
 * output.  Candidates that do not run on the device, or whose bounded barrier waits
 * expire, are skipped.  The fastest is applied to the batch (parameters included).
 * cache_path (host string or NULL): a text file of one line per tuned batch, keyed
 * by the GPU architecture and the batch signature (sorted (devices, colours) pairs of
 * its circuits); a key already in the file is applied without timing (*cached = 1),
 * a new one is appended.  Outputs (each may be NULL): the configuration, the number
 * of candidates timed.  Synchronises the stream.  CS_ENOTSUP if no candidate runs,
 * CS_EINVAL for reps outside 1..100000 or an unwritable cache file. */
cs_status cs_batch_tune(cs_batch *b, const double *W, const double *L, const double *VTH0,
                        const double *x, double ag0, double *A, double *b_vec, int32_t reps,
                        const char *cache_path, cs_batch_config *best, int32_t *n_tried,
                        int32_t *cached, void *stream);

/* One launch over every circuit of the batch. */
cs_status cs_batch_eval_stamp(cs_batch *b, const double *x, double ag0, const double *hist,
                              double *A, double *b_vec, void *stream);
cs_status cs_batch_vjp(cs_batch *b, const double *x, double ag0, const double *hist,
                       const double *A_bar, const double *b_bar, double *W_bar, double *L_bar,
                       double *VTH0_bar, void *stream);
cs_status cs_batch_check(cs_batch *b, void *stream);
/* cs_newton over every circuit of the batch at once (the paper's motivation: a
 * sizing loop simulates many variants of a circuit, Introduction).  The batch's
 * matrix is block diagonal: one solve of the packed system (x, b by rows, A_val by
 * nonzeros in batch order) is one Newton step of every circuit.  Stamping is
 * cs_batch_eval_stamp; the host factorisation (made at the first call on this batch)
 * orders the packed pattern as cs_newton orders one circuit's, each circuit's
 * voltage sources paired within it; node rows of every circuit are clamped.  The
 * iteration stops when the largest step over all circuits is <= tol.  Arguments,
 * outputs and errors as in cs_newton. */
cs_status cs_batch_newton(cs_batch *b, int32_t solver, double *x, double ag0, const double *hist,
                          int32_t max_iter, double vstep, double tol, double *A_val, double *b_vec,
                          int32_t *n_iter, int32_t *converged, double *last_step, double *times_ms,
                          void *stream);

/* Message for the last non-OK status returned to the calling thread. */
const char *cs_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
