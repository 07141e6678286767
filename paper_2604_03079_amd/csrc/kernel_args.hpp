// Plain structs passed from the host launchers to the kernels.
#pragma once
#include <cstdint>

namespace cs {

// Number of stamp-code rows per device: k*k matrix entries plus k RHS entries for
// k <= 4 distinct non-ground nodes.
constexpr int NCODE = 20;

// Stamp codes: bits 30..31 = tag, bits 0..29 = index.
constexpr uint32_t TAG_ADD = 0u;    // load-add into A (or b)
constexpr uint32_t TAG_STORE = 1u;  // plain store (first writer in colour order)
constexpr uint32_t TAG_HUB = 2u;    // store into the hub staging array
constexpr int32_t INDEX_LIMIT = 1 << 30;

// Region schedule codes: tag LDS_ADD / LDS_STORE address the workgroup's LDS
// accumulators, tag STAGE the global staging array (hub and shared-entry
// contributions).  Tag 3 marks an unused code row.
constexpr uint32_t TAG_LDS_ADD = 0u;
constexpr uint32_t TAG_LDS_STORE = 1u;
constexpr uint32_t TAG_STAGE = 2u;
// Targets of region items and interior entries: bits 30..31 = kind.
constexpr uint32_t ITEM_A = 0u;     // A slot
constexpr uint32_t ITEM_B = 1u;     // b row
constexpr uint32_t ITEM_HUB = 2u;   // hub chunk (index = chunk id)
// Per-region table fields: first position, NMOS count, PMOS count (lanes: NMOS
// first, then PMOS), phases, interior range [4], [5) in int_target,
// item range [6], [7) in ritems, lane-fold range [8], [9) in fold, local hub chunk
// range [10], [11) in hfold.
constexpr int FOLD_HEAD = 4;
constexpr int RT_FIELDS = 12;
// A region's items, one int4 per link (ritems entry): item, first staged value,
// target, count | regions << ITEM_NEED_SHIFT, so that a thread's item arrives in one
// round trip.
constexpr int ITEM_NEED_SHIFT = 16;
// Shared entries with more contributions than this are folded by the follow-up
// kernel; smaller ones by the last contributing region, one lane each.
constexpr int ITEM_LANE_MAX = 8;
// An entry whose writers all lie in one region is accumulated in that region's LDS
// by phases only if it has at most this many writers (one or two: two writers need
// only distinct phases, not an order); a larger one is a lane fold: one lane of the
// region folds the writers' merged values, read from LDS in colour order, and
// stores the result.
constexpr int LDS_WRITERS_MAX = 2;
// LDS a region workgroup may use (bytes): owned-entry slots plus merged-value rows.
constexpr int64_t REGION_LDS_LIMIT = 65536 - 1024;
// Staged slots in the grid-barrier form of the region schedule: a shared entry's
// first writer (colour order) stores, the others load-add; hub slots are staged.
constexpr uint8_t SLOT_STORE = 0;
constexpr uint8_t SLOT_ADD = 1;
constexpr uint8_t SLOT_HUB = 2;
constexpr uint8_t SLOT_DEFER = 3;   // large shared entry: staged, folded by the follow-up kernel
constexpr uint32_t HUB_B_FLAG = 0x80000000u;  // hub target is a b row

// Fixed-shape hub sum: the pairwise tree over a hub's contributions in ascending
// device index (padded with -0.0 to a power of two), formed chunk by chunk: each
// aligned chunk of HUB_K contributions is a subtree (one wave), then the chunk sums.
constexpr int HUB_K = 256;
// Largest number of chunks of one hub (the chunk sums are summed by one wave).
constexpr int HUB_MAX_CHUNKS = 2048;
// The region schedule's hub parts: aligned blocks of RHUB_K contributions (also
// subtrees), so that a region of the usual size holds whole parts and sums them from
// its own LDS; a follow-up kernel sums each hub's parts (HUB_K / RHUB_K times as many
// as its chunks).
constexpr int RHUB_K = 32;
constexpr int HUB_MAX_PARTS = HUB_MAX_CHUNKS * (HUB_K / RHUB_K);
// Arrival counters (hub chunks, region items) sit CNT_STRIDE words apart, one per
// 64-byte line: atomics on different words of one line serialise like atomics on one.
constexpr int CNT_STRIDE = 16;

// Per-device constants of the model's bias-dependent part, computed from W, L, VTH0
// and the card when the parameters are set (rows of KCirc::sdp, in DevConstT order).
constexpr int NSD = 10;

// Card-derived constants of the device model, evaluated once on the host in the
// model's operation order.
struct DevCard {
    double VT, COXE, LT, LA, SQPHIS, VBM, NCDEP, INV_TOXE, COXE_KS, TWO_VT, FOUR_DELTA,
        FOUR_DELTA1_VBM, VBI_M_PHIS, K3_TOXE_PHIS, TWO_WINT, TWO_LINT, TWO_VSAT;
    double phis, k1, k2, eta0, nfactor, cdsc, voff, u0, ua, ub, uc, toxe, delta, delta1,
        dvt0, dvt1, dsub, w0, lambda_l, a0, cgdo;
    // source/drain-body junctions (jmod != 0): card values and derived constants
    // (all doubles: the struct has no padding, so cards compare bytewise)
    double jmod;
    double js, cj, pb, hdif, vjmax, NJ_VT, FCPB, FCPB2, TWO_PB, QUARTER_PB, JF1, JF2, JF3;
};

// Device view of one (possibly batched) circuit in colour-major position order.
struct KCirc {
    int32_t n;               // devices
    int32_t n_colors;
    int32_t nc_max;          // largest number of code rows of a device (k*k + k)
    const int32_t *term;     // [4][n]: x index + 1 of d, g, s, b (0 = ground)
    const int8_t *pol;       // [n]
    const double *par;       // [3][n]: W, L, VTH0 (the adjoint's input)
    const double *sdp;       // [NSD][n]: per-device constants of the model (dev_const)
    const int32_t *code;     // [NCODE][n]
    const int32_t *acode;    // [NCODE][n]
    const int32_t *perm;     // [n] position -> caller's device index
    const int32_t *cptr;     // [n_colors+1]
    int32_t n_fixA, n_fixB;
    const int32_t *fixA_idx;
    const double *fixA_val;
    const int32_t *fixB_idx;
    const double *fixB_val;
    int32_t n_hub;
    const int32_t *hub_ptr;      // [n_hub+1] contribution ranges in the staging array
    const int32_t *hub_target;
    double *stage;
    int32_t n_hub_chunks;        // chunks of HUB_K contributions over all hubs
    const int32_t *hub_cptr;     // [n_hub+1] chunk ranges
    const int32_t *hub_of_chunk; // [n_hub_chunks]
    double *hub_part;            // [n_hub_chunks] chunk sums
    uint32_t *hub_count;         // [n_hub * CNT_STRIDE] chunks done (returns to 0 after each call)
    DevCard card[2];         // 0 NMOS, 1 PMOS
};

// Circuits of a batch that are stamped entirely inside one workgroup (colour
// phases separated by workgroup barriers).  table[6*i ..]: first position, last
// position + 1, offset of its colour pointers in cptr, number of colours, first hub
// chunk, last hub chunk + 1.
struct KLocal {
    int32_t n;
    const int32_t *table;
    const int32_t *cptr;
};

// Region schedule (one workgroup per region).
struct KRegion {
    int32_t n_regions;
    const int32_t *rtab;        // [n_regions][RT_FIELDS]
    const uint16_t *phase;      // [n] phase of each position
    const int32_t *int_target;  // interior entries: A slot or b row | ITEM_B<<30, LDS slot = rank
    const int32_t *ritems;      // items each region contributes to
    const int32_t *item;        // [4] per item: first staged value, count, target, regions
                                // (0: folded by the follow-up kernel)
    const int32_t *ritem_head;  // [4] per link: item, first staged value, target,
                                // count | regions << ITEM_NEED_SHIFT
    uint32_t *item_count;       // [items * CNT_STRIDE] arrivals per item (returns to 0 after each call)
    int32_t lds_int;            // LDS doubles reserved for interior entries
    int32_t nc_max;             // largest number of code rows of a device (k*k + k)
    int32_t n_deferred;         // items folded by the follow-up kernel
    const int32_t *deferred;
    // grid-barrier form: shared entries written in place, level by level
    int32_t max_glevel;         // levels of shared-entry writers (-1: beyond 16 bits, form unavailable)
    const uint16_t *glevel;     // [n] level of each position's shared entries
    const int32_t *slot_tgt;    // [staged slots] target of a shared entry
    const uint8_t *slot_first;  // [staged slots] SLOT_STORE / SLOT_ADD / SLOT_HUB / SLOT_DEFER
    // lane folds: [3 per fold] target, first source, count; sources in colour order,
    // each (code row << 16) | lane of a writer in the region
    const int32_t *fold;
    const int32_t *fold_src;
    // per fold its first FOLD_HEAD sources (0 beyond its count), so that a lane's fold
    // and the start of its sources arrive in one round trip
    const int32_t *fold_head;
    // local hub parts: part index of each; the region's k-th local part occupies LDS
    // slots [n_owned + RHUB_K k, n_owned + RHUB_K (k + 1)) after its owned entries,
    // contribution r of the part at slot r
    const int32_t *hfold;
};

// Per-call operands.
struct KCall {
    const double *x;
    double ag0;
    const double *hist;      // caller order [n][4] or nullptr
    double *A;
    double *b;
};

// Grid-barrier state: sync[0] = release epoch, sync[1] = error word,
// sync[2 + blk] = arrival epoch of block blk.
struct KSync {
    uint32_t *sync;
    int64_t spin_limit;
};

}  // namespace cs
