// Internal definitions of the colorstamp library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "colorstamp.h"
#include "kernel_args.hpp"

namespace cs {

// Thread-local error message behind cs_last_error().
void set_error(const std::string &msg);

// Status carrier for internal helpers.
struct Err {
    cs_status st;
    std::string msg;
};

// Owned device allocation.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count) {
        release();
        n = count;
        if (count == 0) return hipSuccess;
        return hipMalloc(reinterpret_cast<void **>(&p), sizeof(T) * count);
    }
    hipError_t upload(const std::vector<T> &h) {
        hipError_t e = alloc(h.size());
        if (e != hipSuccess || h.empty()) return e;
        return hipMemcpy(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
    }
};

// Host-side topology, colouring, pattern and stamp map of one circuit.
struct HostCircuit {
    int32_t n_nodes = 0, n_dev = 0, n_vsrc = 0;
    std::vector<int32_t> term;        // n_dev*4, original order
    std::vector<int8_t> pol;          // n_dev
    std::vector<int32_t> vsrc;        // n_vsrc*2
    std::vector<double> vsrc_volts;   // n_vsrc
    std::vector<int32_t> res;         // 2*n_res: series resistors' nodes (linear, stamped after the FETs)
    std::vector<double> res_g;        // n_res: their conductances

    // colouring
    bool coloured = false;
    std::vector<uint8_t> excl;        // n_nodes (all zero = paper rule)
    int32_t n_colors = 0;
    std::vector<int32_t> colour;      // n_dev
    std::vector<int32_t> perm;        // position -> device (colour-major, stable)
    std::vector<int32_t> colour_ptr;  // n_colors+1

    // pattern and map
    bool mapped = false;
    int32_t n_rows = 0;
    int64_t nnz = 0;
    std::vector<int32_t> row_ptr, col_idx;
    std::vector<int32_t> code;        // NCODE*n_dev, colour-major SoA (tag | index)
    std::vector<int32_t> acode;       // NCODE*n_dev, plain A/b targets (atomic variant)
    std::vector<int32_t> fixA_idx, fixB_idx;
    std::vector<double> fixA_val, fixB_val;
    std::vector<int32_t> linA_idx;    // entries with device writers and a linear part
    std::vector<double> linA_val;     // that part, added after the device contributions
    std::vector<int32_t> hub_ptr;     // n_hub+1 into the staging array
    std::vector<int32_t> hub_target;  // A index, or b row | HUB_B_FLAG
    std::vector<int32_t> hub_cptr;    // n_hub+1: chunk ranges (chunks of HUB_K)
    std::vector<int32_t> hub_of_chunk;
    int32_t max_hub_len = 0;
    int32_t max_nc = 0;               // largest k*k + k over the devices
};

// Input of the region planner: a colour-major table (single circuit or packed batch).
struct RegionSource {
    int32_t n = 0;                         // positions
    std::vector<int32_t> code;             // [NCODE][n] tags ADD/STORE/HUB
    std::vector<int32_t> term;             // [4][n] x index + 1
    std::vector<int8_t> pol;               // [n]
    std::vector<int32_t> perm;             // position -> global device index
    std::vector<int32_t> colour;           // [n] colour of each position (within its circuit)
    std::vector<int64_t> group_ptr;        // circuit boundaries over global devices (empty: one)
    int64_t nnz = 0, n_rows = 0;
    std::vector<int32_t> hub_ptr, hub_cptr;
    int64_t stage_base = 0;                // hub staging size; shared entries staged after it
    int32_t cus = 0;                       // compute units of the target GPU (0: unknown)
};

// Region schedule tables (host), region-major positions.
struct RegionPlan {
    bool built = false;
    int32_t cap = 0, n_regions = 0, max_lds = 0, max_phase = 0, max_nc = 0, max_glevel = 0, cus = 0;
    int64_t stage_size = 0;
    std::vector<int32_t> perm, cm_pos, term, code, rtab, int_target, ritems, item, deferred;
    std::vector<int8_t> pol;
    std::vector<uint16_t> phase, glevel;
    std::vector<int32_t> slot_tgt;     // per staged slot: target of a shared entry (-1: hub)
    std::vector<uint8_t> slot_first;   // SLOT_STORE / SLOT_ADD / SLOT_HUB / SLOT_DEFER
    std::vector<int32_t> fold, fold_src;   // lane folds (see KRegion)
    // hub parts of the region schedule: chunks of RHUB_K contributions
    std::vector<int32_t> hub_cptr;         // n_hub+1: part ranges per hub
    std::vector<int32_t> hub_of_chunk;     // hub of each part
    std::vector<int32_t> hfold;            // local hub parts (see KRegion)
};

// Device copies of a region plan.
struct RegionDev {
    DevBuf<int32_t> perm, cm_pos, term, code, rtab, int_target, ritems, item, deferred;
    DevBuf<int8_t> pol;
    DevBuf<uint16_t> phase, glevel;
    DevBuf<int32_t> slot_tgt;
    DevBuf<uint8_t> slot_first;
    DevBuf<int32_t> fold, fold_src;
    DevBuf<int32_t> fold_head;   // per fold its first FOLD_HEAD sources (0 beyond its count)
    DevBuf<int32_t> ritem_head;  // per link its item's fields (KRegion::ritem_head)
    DevBuf<int32_t> hub_cptr, hub_of_chunk, hfold;
    DevBuf<double> hub_part;
    DevBuf<double> sdp, stage;   // sdp: per-device model constants, region-major [NSD][n]
    DevBuf<uint32_t> item_count;
    bool ready = false;      // uploaded from the current plan
    bool sdp_stale = true;
};

Err build_regions(const RegionSource &s, int32_t cap, RegionPlan &R);
hipError_t upload_regions(const RegionPlan &R, RegionDev &D);
// Kernel views of the region tables: base supplies the fixed stores and hub tables.
KCirc region_kcirc(const KCirc &base, const RegionPlan &R, const RegionDev &D);
KRegion region_kregion(const RegionPlan &R, const RegionDev &D);
void region_info(const RegionPlan &R, int32_t *n_regions, int32_t *max_phases, int64_t *n_items,
                 int64_t *n_staged, int64_t *n_interior, int64_t *n_links, int64_t *n_folds,
                 int64_t *n_fold_src);
void region_tables(const RegionPlan &R, int32_t *perm, uint16_t *phase, int32_t *code, int32_t *rtab,
                   int32_t *interior, int32_t *links, int32_t *item, int32_t *fold, int32_t *fold_src);
void region_hub_tables(const RegionPlan &R, int64_t *counts, int32_t *hfold, int32_t *part_ptr);

// Build the greedy colouring (ascending device order) and the colour-major order.
// order: 0 ascending device index (the paper's), 1 largest degree first, 2 DSATUR.
Err build_colouring(HostCircuit &h, const uint8_t *exclude, int64_t *n_edges, int order = 0);
// Build pattern, stamp codes, fixed stores and hub lists.
Err build_map(HostCircuit &h);
// Card-derived constants, in the model's operation order.
DevCard derive_card(const cs_model_card &c);

// Sparse LU of P A Q: row order P (P[k] = row pivoted at step k), column order Q,
// and the bundle T = (L - I) + U in CSR over the permuted indices.
struct HostLU {
    std::vector<int32_t> P, Q, Tp, Ti;
    std::vector<double> Tx;
};
// An MNA matrix pattern for the sparse solve: n rows, CSR, and per voltage source
// its two terminal node rows (-1 for ground) and its branch row.
struct MnaView {
    int32_t n = 0;
    const int32_t *row_ptr = nullptr, *col_idx = nullptr;
    std::vector<std::array<int32_t, 3>> src;
};
MnaView circuit_view(const HostCircuit &h);
// Column order Q (source pairs first, then nested dissection (method 0) or minimum
// degree (method 1)) and the preferred pivot row of each column (-1: its own row).
void mna_order(const MnaView &m, std::vector<int32_t> &Q, std::vector<int32_t> &pref, int method);
// Factor with both orders, keep the one with the lower estimated level-scheduled cost.
Err factor_mna(const MnaView &m, const double *A, HostLU &F, int *method);
// One factorisation with threshold partial pivoting (host values of A in CSR).
Err host_lu(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
            const std::vector<int32_t> &Q, const std::vector<int32_t> &pref, HostLU &F);

// GPU state of the Newton loop (solver handles, factor pattern); released with the circuit.
struct NewtonState;
void destroy_newton(NewtonState *s);

}  // namespace cs

struct cs_circuit {
    cs::HostCircuit h;
    bool models_set = false;
    bool params_set = false;
    cs::DevCard card[2];               // 0 NMOS, 1 PMOS
    int device = -1;                   // HIP device of the uploads
    // device copies (colour-major)
    cs::DevBuf<int32_t> d_term, d_code, d_acode, d_perm, d_cptr, d_fixA_idx, d_fixB_idx,
        d_hub_ptr, d_hub_target, d_hub_cptr, d_hub_of_chunk;
    cs::DevBuf<int8_t> d_pol;
    cs::DevBuf<double> d_par, d_fixA_val, d_fixB_val, d_stage, d_buf, d_hub_part;
    cs::DevBuf<double> d_sdp;          // per-device model constants [NSD][n] (colour-major)
    cs::DevBuf<int32_t> d_linA_idx;
    cs::DevBuf<double> d_linA_val;
    cs::DevBuf<int32_t> d_ipos;   // device index -> position (serial stamping)
    cs::DevBuf<uint32_t> d_sync;       // barrier words + per-block arrival flags + error
    cs::DevBuf<uint32_t> d_hub_count;
    int32_t block = 256;
    int32_t eval_ahead_req = -1;
    bool cooperative = true;
    int32_t grid = 0;                  // persistent grid
    int32_t eval_ahead = 0;
    int64_t spin_limit = 1 << 22;
    int32_t grid_key = 0;              // which plan c->grid belongs to
    cs::RegionPlan rp;                 // region schedule (built on first use, per block size)
    cs::RegionDev rd;
    int32_t rg_cap_block = 0, rg_cap_regions = -1;   // resident-region capacity cache
    int32_t plan_cus = -1;   // compute units the region planner targets (-1: the current GPU's)
    int64_t rg_cap = 0;
    cs::NewtonState *newton = nullptr;   // built by the first cs_newton on this stamp map
    int32_t newton_flags = 0;             // CS_NEWTON_NO_* bits of cs_set_newton_options
    cs_circuit() = default;
    cs_circuit(const cs_circuit &) = delete;
    cs_circuit &operator=(const cs_circuit &) = delete;
    ~cs_circuit() { cs::destroy_newton(newton); }
};

namespace cs {
// Kernel view of a single circuit's device copies (colour-major).
KCirc make_kcirc(cs_circuit *c);
}  // namespace cs

struct cs_batch {
    std::vector<cs_circuit *> circ;
    std::vector<int64_t> dev_off, row_off, nnz_off;   // n+1 each
    cs::DevCard card[2];
    // packed instance table (built for the current local_max_dev)
    bool packed = false;
    bool params_set = false;
    cs::HostCircuit h;                 // packed codes, permutation, colour pointers, hubs
    std::vector<int32_t> pterm;        // [4][positions] x index + 1
    std::vector<int8_t> ppol;
    std::vector<int32_t> pcolour;      // colour of each packed position (within its circuit)
    std::vector<int32_t> local_table;  // 6 per workgroup-local circuit
    std::vector<int32_t> local_cptr;
    int32_t n_local = 0;
    int32_t n_global_chunks = 0;
    int64_t stage_total = 0;
    // device copies
    int device = -1;
    cs::DevBuf<int32_t> d_term, d_code, d_acode, d_perm, d_cptr, d_fixA_idx, d_fixB_idx,
        d_hub_ptr, d_hub_target, d_hub_cptr, d_hub_of_chunk, d_local, d_local_cptr;
    cs::DevBuf<int8_t> d_pol;
    cs::DevBuf<double> d_par, d_fixA_val, d_fixB_val, d_stage, d_hub_part;
    cs::DevBuf<double> d_sdp;          // per-device model constants [NSD][n] (packed order)
    cs::DevBuf<int32_t> d_linA_idx;
    cs::DevBuf<double> d_linA_val;
    cs::DevBuf<uint32_t> d_sync, d_hub_count;
    // launch
    int32_t block = 256;
    int32_t eval_ahead_req = -1;
    int32_t local_max_dev = 0;
    bool cooperative = true;
    int32_t grid = 0, n_part = 0, eval_ahead = 0;
    int64_t spin_limit = 1 << 22;
    cs_variant schedule = CS_COLOR_PERSISTENT;
    cs::RegionPlan rp;
    cs::RegionDev rd;
    // Newton loop state (block-diagonal pattern, built by the first cs_batch_newton)
    std::vector<int32_t> nt_row_ptr, nt_col_idx;
    cs::NewtonState *newton = nullptr;
    cs_batch() = default;
    cs_batch(const cs_batch &) = delete;
    cs_batch &operator=(const cs_batch &) = delete;
    ~cs_batch() { cs::destroy_newton(newton); }
};
