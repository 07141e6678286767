// Batches of independent circuits stamped in one launch, and the adjoint entry points.
//
// A batch is packed as one block-diagonal instance table: per-circuit node, row,
// nonzero and hub-staging indices are offset into packed arrays (x and b by rows, A
// by nonzeros).  Circuits with more devices than local_max_dev follow the
// grid-barrier colour schedule (colour c of every such circuit forms global phase
// c); the others are stamped entirely inside one workgroup each, their colour phases
// separated by workgroup barriers (colour-phase fusion).  Every circuit keeps its
// own colouring and its own colour order, so the result equals the per-circuit one.
#include <algorithm>
#include <cstring>
#include <new>

#include "colorstamp.h"
#include "internal.hpp"
#include "launch.hpp"

using namespace cs;

namespace {

cs_status bfail(cs_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

#define CS_BCHECK(expr, what)                                                          \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return bfail(CS_EHIP, std::string(what) + ": " + hipGetErrorString(e_)); \
    } while (0)

int cur_device() {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return -1;
    return d;
}

int distinct_nodes(const int32_t *t) {
    int k = 0;
    for (int i = 0; i < 4; ++i) {
        if (t[i] == 0) continue;
        bool seen = false;
        for (int j = 0; j < i; ++j) seen = seen || t[j] == t[i];
        if (!seen) ++k;
    }
    return k;
}

// Build the packed instance table for the current local_max_dev.
cs_status pack(cs_batch *B) {
    const size_t nc = B->circ.size();
    std::vector<size_t> glob, loc;
    int32_t cmax = 0;
    for (size_t i = 0; i < nc; ++i) {
        const HostCircuit &h = B->circ[i]->h;
        if (h.n_dev > B->local_max_dev) {
            glob.push_back(i);
            cmax = std::max(cmax, h.n_colors);
        } else if (h.n_dev > 0 || !h.hub_target.empty()) {
            loc.push_back(i);
        }
    }
    // staging ranges in hub order: global circuits first, then local ones, so that
    // every hub's contributions are contiguous and the global hubs come first
    std::vector<int64_t> stage_off(nc, 0);
    int64_t stage_total = 0;
    for (size_t i : glob) { stage_off[i] = stage_total; stage_total += B->circ[i]->h.hub_ptr.empty() ? 0 : B->circ[i]->h.hub_ptr.back(); }
    for (size_t i : loc) { stage_off[i] = stage_total; stage_total += B->circ[i]->h.hub_ptr.empty() ? 0 : B->circ[i]->h.hub_ptr.back(); }
    if (B->nnz_off[nc] >= INDEX_LIMIT || B->row_off[nc] >= INDEX_LIMIT || stage_total >= INDEX_LIMIT)
        return bfail(CS_ENOTSUP, "batch too large for 30-bit stamp codes");
    const int64_t n_pos = B->dev_off[nc];
    HostCircuit &P = B->h;
    P.n_dev = (int32_t)n_pos;
    P.n_colors = cmax;
    P.max_nc = 0;
    for (size_t i = 0; i < nc; ++i) P.max_nc = std::max(P.max_nc, B->circ[i]->h.max_nc);
    P.perm.assign((size_t)n_pos, 0);
    P.colour_ptr.assign((size_t)cmax + 1, 0);
    std::vector<std::pair<int32_t, int32_t>> src;   // (circuit, position) per packed position
    src.reserve((size_t)n_pos);
    for (int32_t c = 0; c < cmax; ++c) {
        for (size_t i : glob) {
            const HostCircuit &h = B->circ[i]->h;
            if (c >= h.n_colors) continue;
            for (int32_t p = h.colour_ptr[(size_t)c]; p < h.colour_ptr[(size_t)c + 1]; ++p)
                src.emplace_back((int32_t)i, p);
        }
        P.colour_ptr[(size_t)c + 1] = (int32_t)src.size();
    }
    B->local_table.clear();
    B->local_cptr.clear();
    for (size_t i : loc) {
        const HostCircuit &h = B->circ[i]->h;
        const int32_t first = (int32_t)src.size();
        for (int32_t p = 0; p < h.n_dev; ++p) src.emplace_back((int32_t)i, p);
        B->local_table.insert(B->local_table.end(),
                              {first, (int32_t)src.size(), (int32_t)B->local_cptr.size(), h.n_colors, 0, 0});
        for (int32_t c = 0; c <= h.n_colors; ++c) B->local_cptr.push_back(first + h.colour_ptr[(size_t)c]);
    }
    const size_t n = (size_t)n_pos;
    B->pterm.assign(4 * n, 0);
    B->ppol.assign(n, 0);
    B->pcolour.assign(n, 0);
    B->rp = RegionPlan{};
    B->rd.ready = false;
    P.code.assign((size_t)NCODE * n, 0);
    P.acode.assign((size_t)NCODE * n, 0);
    for (size_t q = 0; q < n; ++q) {
        const int32_t i = src[q].first, p = src[q].second;
        const HostCircuit &h = B->circ[(size_t)i]->h;
        const size_t ni = (size_t)h.n_dev;
        const int32_t v = h.perm[(size_t)p];
        const int32_t *t4 = &h.term[4 * (size_t)v];
        for (int j = 0; j < 4; ++j)
            B->pterm[(size_t)j * n + q] = t4[j] == 0 ? 0 : (int32_t)(B->row_off[(size_t)i] + t4[j]);
        B->ppol[q] = h.pol[(size_t)v];
        B->pcolour[q] = h.colour[(size_t)v];
        P.perm[q] = (int32_t)(B->dev_off[(size_t)i] + v);
        const int k = distinct_nodes(t4);
        for (int j = 0; j < k * k + k; ++j) {
            const uint32_t c = (uint32_t)h.code[(size_t)j * ni + (size_t)p];
            const uint32_t tag = c >> 30;
            uint32_t idx = c & 0x3FFFFFFFu;
            if (tag == TAG_HUB) idx += (uint32_t)stage_off[(size_t)i];
            else idx += (uint32_t)(j < k * k ? B->nnz_off[(size_t)i] : B->row_off[(size_t)i]);
            P.code[(size_t)j * n + q] = (int32_t)((tag << 30) | idx);
            P.acode[(size_t)j * n + q] = h.acode[(size_t)j * ni + (size_t)p] +
                                         (int32_t)(j < k * k ? B->nnz_off[(size_t)i] : B->row_off[(size_t)i]);
        }
    }
    // fixed stores
    P.fixA_idx.clear(); P.fixA_val.clear(); P.fixB_idx.clear(); P.fixB_val.clear();
    for (size_t i = 0; i < nc; ++i) {
        const HostCircuit &h = B->circ[i]->h;
        for (size_t e = 0; e < h.fixA_idx.size(); ++e) {
            P.fixA_idx.push_back((int32_t)(h.fixA_idx[e] + B->nnz_off[i]));
            P.fixA_val.push_back(h.fixA_val[e]);
        }
        for (size_t e = 0; e < h.fixB_idx.size(); ++e) {
            P.fixB_idx.push_back((int32_t)(h.fixB_idx[e] + B->row_off[i]));
            P.fixB_val.push_back(h.fixB_val[e]);
        }
    }
    // linear parts of the circuits' series resistors
    P.linA_idx.clear(); P.linA_val.clear();
    for (size_t i = 0; i < nc; ++i) {
        const HostCircuit &h = B->circ[i]->h;
        for (size_t e = 0; e < h.linA_idx.size(); ++e) {
            P.linA_idx.push_back((int32_t)(h.linA_idx[e] + B->nnz_off[i]));
            P.linA_val.push_back(h.linA_val[e]);
        }
    }
    // hubs: global circuits first (their chunks form the global hub phase), then
    // each local circuit's own chunk range
    P.hub_ptr.assign(1, 0);
    P.hub_target.clear();
    P.hub_cptr.assign(1, 0);
    P.hub_of_chunk.clear();
    auto add_hubs = [&](size_t i) {
        const HostCircuit &h = B->circ[i]->h;
        for (size_t k = 0; k + 1 < h.hub_ptr.size(); ++k) {
            const int32_t m = h.hub_ptr[k + 1] - h.hub_ptr[k];
            P.hub_ptr.push_back((int32_t)(stage_off[i] + h.hub_ptr[k + 1]));
            const uint32_t tg = (uint32_t)h.hub_target[k];
            P.hub_target.push_back((tg & HUB_B_FLAG)
                                       ? (int32_t)((uint32_t)((tg & ~HUB_B_FLAG) + B->row_off[i]) | HUB_B_FLAG)
                                       : (int32_t)(tg + B->nnz_off[i]));
            const int32_t ncnk = (m + HUB_K - 1) / HUB_K;
            for (int32_t j = 0; j < ncnk; ++j) P.hub_of_chunk.push_back((int32_t)P.hub_target.size() - 1);
            P.hub_cptr.push_back(P.hub_cptr.back() + ncnk);
        }
    };
    for (size_t i : glob) add_hubs(i);
    B->n_global_chunks = (int32_t)P.hub_of_chunk.size();
    for (size_t li = 0; li < loc.size(); ++li) {
        B->local_table[6 * li + 4] = (int32_t)P.hub_of_chunk.size();
        add_hubs(loc[li]);
        B->local_table[6 * li + 5] = (int32_t)P.hub_of_chunk.size();
    }
    B->n_local = (int32_t)loc.size();
    B->stage_total = stage_total;
    B->packed = true;
    return CS_OK;
}

cs_status upload(cs_batch *B) {
    HostCircuit &P = B->h;
    CS_BCHECK(B->d_term.upload(B->pterm), "upload terminals");
    CS_BCHECK(B->d_pol.upload(B->ppol), "upload polarity");
    CS_BCHECK(B->d_code.upload(P.code), "upload codes");
    CS_BCHECK(B->d_acode.upload(P.acode), "upload codes");
    CS_BCHECK(B->d_perm.upload(P.perm), "upload permutation");
    CS_BCHECK(B->d_cptr.upload(P.colour_ptr), "upload colour pointers");
    CS_BCHECK(B->d_fixA_idx.upload(P.fixA_idx), "upload fixed stores");
    CS_BCHECK(B->d_fixA_val.upload(P.fixA_val), "upload fixed stores");
    CS_BCHECK(B->d_fixB_idx.upload(P.fixB_idx), "upload fixed stores");
    CS_BCHECK(B->d_fixB_val.upload(P.fixB_val), "upload fixed stores");
    CS_BCHECK(B->d_linA_idx.upload(P.linA_idx), "upload linear part");
    CS_BCHECK(B->d_linA_val.upload(P.linA_val), "upload linear part");
    CS_BCHECK(B->d_hub_ptr.upload(P.hub_ptr), "upload hubs");
    CS_BCHECK(B->d_hub_target.upload(P.hub_target), "upload hubs");
    CS_BCHECK(B->d_hub_cptr.upload(P.hub_cptr), "upload hubs");
    CS_BCHECK(B->d_hub_of_chunk.upload(P.hub_of_chunk), "upload hubs");
    CS_BCHECK(B->d_stage.alloc((size_t)B->stage_total), "alloc staging");
    CS_BCHECK(B->d_hub_part.alloc(P.hub_of_chunk.size()), "alloc hub partials");
    CS_BCHECK(B->d_hub_count.alloc(P.hub_target.size() * CNT_STRIDE), "alloc hub counters");
    if (!P.hub_target.empty())
        CS_BCHECK(hipMemset(B->d_hub_count.p, 0, sizeof(uint32_t) * B->d_hub_count.n), "clear hub counters");
    CS_BCHECK(B->d_local.upload(B->local_table), "upload local table");
    CS_BCHECK(B->d_local_cptr.upload(B->local_cptr), "upload local table");
    if (B->d_par.n < 3 * (size_t)P.n_dev) CS_BCHECK(B->d_par.alloc(3 * (size_t)P.n_dev), "alloc parameters");
    if (B->d_sdp.n < (size_t)NSD * P.n_dev) CS_BCHECK(B->d_sdp.alloc((size_t)NSD * P.n_dev), "alloc model constants");
    if (B->d_sync.n == 0) {
        hipDeviceProp_t prop;
        CS_BCHECK(hipGetDeviceProperties(&prop, cur_device()), "device properties");
        const size_t words = 2 + (size_t)prop.multiProcessorCount * 64;
        CS_BCHECK(B->d_sync.alloc(words), "alloc barrier state");
        CS_BCHECK(hipMemset(B->d_sync.p, 0, words * sizeof(uint32_t)), "clear barrier state");
    }
    B->device = cur_device();
    B->grid = 0;
    return CS_OK;
}

KCirc make_kc(cs_batch *B) {
    KCirc k{};
    const HostCircuit &P = B->h;
    k.n = P.n_dev;
    k.n_colors = P.n_colors;
    k.nc_max = P.max_nc;
    k.term = B->d_term.p;
    k.pol = B->d_pol.p;
    k.par = B->d_par.p;
    k.sdp = B->d_sdp.p;
    k.code = B->d_code.p;
    k.acode = B->d_acode.p;
    k.perm = B->d_perm.p;
    k.cptr = B->d_cptr.p;
    k.n_fixA = (int32_t)P.fixA_idx.size();
    k.n_fixB = (int32_t)P.fixB_idx.size();
    k.fixA_idx = B->d_fixA_idx.p;
    k.fixA_val = B->d_fixA_val.p;
    k.fixB_idx = B->d_fixB_idx.p;
    k.fixB_val = B->d_fixB_val.p;
    k.n_hub = (int32_t)P.hub_target.size();
    k.hub_ptr = B->d_hub_ptr.p;
    k.hub_target = B->d_hub_target.p;
    k.stage = B->d_stage.p;
    k.n_hub_chunks = (int32_t)P.hub_of_chunk.size();
    k.hub_cptr = B->d_hub_cptr.p;
    k.hub_of_chunk = B->d_hub_of_chunk.p;
    k.hub_part = B->d_hub_part.p;
    k.hub_count = B->d_hub_count.p;
    k.card[0] = B->card[0];
    k.card[1] = B->card[1];
    return k;
}

// Split of the persistent grid between the global schedule and the local circuits.
cs_status plan(cs_batch *B) {
    if (B->grid > 0) return CS_OK;
    hipDeviceProp_t prop;
    CS_BCHECK(hipGetDeviceProperties(&prop, B->device), "device properties");
    const int block = B->block;
    int per_cu_ahead = 0, per_cu_phase = 0;
    CS_BCHECK(persistent_capacity(1, block, B->h.max_nc, &per_cu_ahead), "occupancy");
    CS_BCHECK(persistent_capacity(0, block, B->h.max_nc, &per_cu_phase), "occupancy");
    const HostCircuit &P = B->h;
    const int64_t n_sched = P.colour_ptr.empty() ? 0 : P.colour_ptr.back();
    int64_t max_colour = 0;
    for (int32_t k = 0; k < P.n_colors; ++k)
        max_colour = std::max<int64_t>(max_colour, P.colour_ptr[k + 1] - P.colour_ptr[k]);
    const int64_t local_dev = P.n_dev - n_sched;
    const int64_t cap_phase = (int64_t)per_cu_phase * prop.multiProcessorCount;
    const int64_t cap_ahead = (int64_t)per_cu_ahead * prop.multiProcessorCount;
    // workgroups for the local circuits: each runs its colour phases at the latency
    // of one small evaluation, so their count (not their share of devices) sets the
    // time: at least an eighth of the resident workgroups, one per circuit at most
    int64_t n_lb = 0;
    if (B->n_local > 0) {
        n_lb = n_sched == 0 ? std::min<int64_t>(cap_phase, B->n_local)
                            : std::max<int64_t>({(int64_t)1, cap_phase / 8,
                                                 (int64_t)((double)cap_phase * (double)local_dev / (double)P.n_dev)});
        n_lb = std::min<int64_t>(n_lb, B->n_local);
    }
    const int64_t need_ahead = (n_sched + block - 1) / block;
    const bool fits = n_sched > 0 && need_ahead + n_lb <= cap_ahead;
    if (B->eval_ahead_req == 1 && !fits) return bfail(CS_ENOTSUP, "evaluate-ahead needs one resident thread per device");
    B->eval_ahead = B->eval_ahead_req == 0 ? 0 : (fits ? 1 : 0);
    int64_t n_gb = 0;
    if (n_sched > 0) {
        n_gb = B->eval_ahead ? need_ahead
                             : std::max<int64_t>(1, std::min<int64_t>(cap_phase - n_lb, (max_colour + block - 1) / block));
    }
    if (n_gb + n_lb < 1) n_gb = 1;   // fixed stores still need one block
    if (n_gb + n_lb > (B->eval_ahead ? cap_ahead : cap_phase))
        return bfail(CS_ENOTSUP, "batch grid does not fit the device");
    if ((size_t)n_gb + 2 > B->d_sync.n) return bfail(CS_ENOTSUP, "grid larger than the barrier state");
    B->n_part = (int32_t)n_gb;
    B->grid = (int32_t)(n_gb + n_lb);
    return CS_OK;
}

cs_status plan_regions(cs_batch *B, int32_t block) {
    if (B->rp.built && B->rp.cap == block) return CS_OK;
    B->rd.ready = false;
    HostCircuit &P = B->h;
    try {
        RegionSource src;
        src.n = P.n_dev;
        src.code = P.code;
        src.term = B->pterm;
        src.pol = B->ppol;
        src.perm = P.perm;
        src.colour = B->pcolour;
        src.group_ptr = B->dev_off;
        src.nnz = B->nnz_off.back();
        src.n_rows = B->row_off.back();
        src.hub_ptr = P.hub_ptr;
        src.hub_cptr = P.hub_cptr;
        src.stage_base = B->stage_total;
        Err e = build_regions(src, block, B->rp);
        if (e.st == CS_OK && region_lds_bytes(B->rp.max_lds + 1, B->rp.max_nc, block) > (size_t)REGION_LDS_LIMIT)
            e = {CS_ENOTSUP, "region LDS exceeds 64 KiB; use a smaller block"};
        if (e.st != CS_OK) {
            B->rp = RegionPlan{};
            return bfail(e.st, e.msg);
        }
    } catch (const std::bad_alloc &) {
        B->rp = RegionPlan{};
        return bfail(CS_ENOMEM, "host allocation");
    }
    return CS_OK;
}

cs_status ensure_region(cs_batch *B, hipStream_t s) {
    cs_status st = plan_regions(B, B->block);
    if (st != CS_OK) return st;
    if (!B->rd.ready) {
        hipError_t e = upload_regions(B->rp, B->rd);
        if (e != hipSuccess) {
            B->rd.ready = false;
            return bfail(CS_EHIP, std::string("upload region tables: ") + hipGetErrorString(e));
        }
    }
    if (B->rd.sdp_stale) {
        CS_BCHECK(launch_permute_rows(B->h.n_dev, B->rd.cm_pos.p, B->d_sdp.p, B->h.n_dev, NSD, B->rd.sdp.p, s),
                  "model-constant permute launch");
        B->rd.sdp_stale = false;
    }
    return CS_OK;
}

}  // namespace

extern "C" {

cs_status cs_vjp(cs_circuit *c, const double *x, double ag0, const double *hist,
                 const double *A_bar, const double *b_bar, double *W_bar, double *L_bar,
                 double *VTH0_bar, void *stream) {
    if (!c) return bfail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return bfail(CS_ESTATE, "cs_build_stamp_map must come first");
    if (!c->models_set || !c->params_set) return bfail(CS_ESTATE, "models and parameters must be set first");
    if (!x || !A_bar || !b_bar || !W_bar || !L_bar || !VTH0_bar) return bfail(CS_EINVAL, "NULL argument");
    if (cur_device() != c->device) return bfail(CS_ESTATE, "circuit uploaded to another device");
    KCirc kc{};
    kc.n = c->h.n_dev;
    kc.term = c->d_term.p;
    kc.pol = c->d_pol.p;
    kc.par = c->d_par.p;
    kc.acode = c->d_acode.p;
    kc.perm = c->d_perm.p;
    kc.card[0] = c->card[0];
    kc.card[1] = c->card[1];
    const KCall call{x, ag0, hist, nullptr, nullptr};
    CS_BCHECK(launch_vjp(kc, call, A_bar, b_bar, W_bar, L_bar, VTH0_bar, (hipStream_t)stream), "vjp launch");
    return CS_OK;
}

cs_status cs_batch_create(int32_t n, cs_circuit *const *circuits, cs_batch **out) {
    if (!out) return bfail(CS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !circuits) return bfail(CS_EINVAL, "empty batch");
    for (int32_t i = 0; i < n; ++i) {
        const cs_circuit *c = circuits[i];
        if (!c) return bfail(CS_EINVAL, "NULL circuit in batch");
        if (!c->h.mapped || !c->models_set) return bfail(CS_ESTATE, "batch circuits must be mapped and have models");
        if (std::memcmp(&c->card[0], &circuits[0]->card[0], sizeof(DevCard)) ||
            std::memcmp(&c->card[1], &circuits[0]->card[1], sizeof(DevCard)))
            return bfail(CS_ENOTSUP, "batch circuits must share their model cards");
    }
    cs_batch *B = new (std::nothrow) cs_batch();
    if (!B) return bfail(CS_ENOMEM, "host allocation");
    try {
        B->circ.assign(circuits, circuits + n);
        B->dev_off.assign((size_t)n + 1, 0);
        B->row_off.assign((size_t)n + 1, 0);
        B->nnz_off.assign((size_t)n + 1, 0);
        for (int32_t i = 0; i < n; ++i) {
            B->dev_off[(size_t)i + 1] = B->dev_off[(size_t)i] + circuits[i]->h.n_dev;
            B->row_off[(size_t)i + 1] = B->row_off[(size_t)i] + circuits[i]->h.n_rows;
            B->nnz_off[(size_t)i + 1] = B->nnz_off[(size_t)i] + circuits[i]->h.nnz;
        }
    } catch (...) {
        delete B;
        return bfail(CS_ENOMEM, "host allocation");
    }
    if (B->dev_off.back() * NCODE >= ((int64_t)1 << 31)) {
        delete B;
        return bfail(CS_ENOTSUP, "too many devices in the batch");
    }
    B->card[0] = circuits[0]->card[0];
    B->card[1] = circuits[0]->card[1];
    *out = B;
    return CS_OK;
}

void cs_batch_destroy(cs_batch *b) { delete b; }

cs_status cs_batch_layout(const cs_batch *B, int64_t *dev_off, int64_t *row_off, int64_t *nnz_off) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    const size_t n = B->circ.size() + 1;
    if (dev_off) std::memcpy(dev_off, B->dev_off.data(), n * sizeof(int64_t));
    if (row_off) std::memcpy(row_off, B->row_off.data(), n * sizeof(int64_t));
    if (nnz_off) std::memcpy(nnz_off, B->nnz_off.data(), n * sizeof(int64_t));
    return CS_OK;
}

cs_status cs_batch_set_launch(cs_batch *B, int32_t block, int32_t eval_ahead, int32_t local_max_dev) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (block != 0 && (block < 64 || block > 256 || block % 64 != 0))
        return bfail(CS_EINVAL, "block must be 64, 128, 192 or 256");
    if (eval_ahead < -1 || eval_ahead > 1) return bfail(CS_EINVAL, "eval_ahead must be -1, 0 or 1");
    if (local_max_dev < 0) return bfail(CS_EINVAL, "local_max_dev must be >= 0");
    B->block = block ? block : 256;
    B->eval_ahead_req = eval_ahead;
    if (local_max_dev != B->local_max_dev) {
        B->local_max_dev = local_max_dev;
        B->packed = false;
        B->device = -1;
        B->params_set = false;
    }
    B->grid = 0;
    return CS_OK;
}

cs_status cs_batch_set_params(cs_batch *B, const double *W, const double *L, const double *VTH0,
                              void *stream) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (!B->packed) {
        try {
            cs_status st = pack(B);
            if (st != CS_OK) return st;
        } catch (const std::bad_alloc &) {
            return bfail(CS_ENOMEM, "host allocation");
        }
    }
    if (B->device < 0) {
        cs_status st = upload(B);
        if (st != CS_OK) return st;
    }
    if (B->h.n_dev > 0 && (!W || !L || !VTH0)) return bfail(CS_EINVAL, "NULL parameter array");
    if (cur_device() != B->device) return bfail(CS_ESTATE, "batch uploaded to another device");
    CS_BCHECK(launch_gather_params(B->h.n_dev, B->d_perm.p, W, L, VTH0, B->d_par.p, (hipStream_t)stream),
              "parameter gather launch");
    B->params_set = true;
    // per-device model constants, and their region-major copy, on the same stream (a
    // replayed step runs no host code)
    CS_BCHECK(launch_dev_const(make_kc(B), B->d_sdp.p, (hipStream_t)stream), "model-constant launch");
    if (B->rd.ready) {
        CS_BCHECK(launch_permute_rows(B->h.n_dev, B->rd.cm_pos.p, B->d_sdp.p, B->h.n_dev, NSD, B->rd.sdp.p,
                                      (hipStream_t)stream), "model-constant permute launch");
        B->rd.sdp_stale = false;
    } else {
        B->rd.sdp_stale = true;
    }
    return CS_OK;
}

cs_status cs_batch_get_info(const cs_batch *B, int64_t *n_dev, int64_t *n_rows, int64_t *nnz,
                            int32_t *max_colors, int32_t *grid, int32_t *block, int32_t *eval_ahead,
                            int32_t *n_local) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (n_dev) *n_dev = B->dev_off.back();
    if (n_rows) *n_rows = B->row_off.back();
    if (nnz) *nnz = B->nnz_off.back();
    if (max_colors) *max_colors = B->h.n_colors;
    if (grid) *grid = B->grid;
    if (block) *block = B->block;
    if (eval_ahead) *eval_ahead = B->eval_ahead;
    if (n_local) *n_local = B->n_local;
    return CS_OK;
}

cs_status cs_batch_eval_stamp(cs_batch *B, const double *x, double ag0, const double *hist,
                              double *A, double *b_vec, void *stream) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (!B->params_set) return bfail(CS_ESTATE, "cs_batch_set_params must come first");
    if (!x || !A || !b_vec) return bfail(CS_EINVAL, "NULL x, A or b");
    if (cur_device() != B->device) return bfail(CS_ESTATE, "batch uploaded to another device");
    const KCall call{x, ag0, hist, A, b_vec};
    if (B->schedule == CS_COLOR_REGION) {
        cs_status st = ensure_region(B, (hipStream_t)stream);
        if (st != CS_OK) return st;
        const KCirc kc = make_kc(B);
        CS_BCHECK(launch_region(region_kcirc(kc, B->rp, B->rd), call, region_kregion(B->rp, B->rd), B->block,
                                (hipStream_t)stream), "batched region launch");
    } else {
        cs_status st = plan(B);
        if (st != CS_OK) return st;
        const KCirc kc = make_kc(B);
        const KSync ks{B->d_sync.p, B->spin_limit};
        const KLocal kl{B->n_local, B->d_local.p, B->d_local_cptr.p};
        CS_BCHECK(launch_persistent(kc, call, ks, nullptr, B->eval_ahead, B->grid, B->block, B->cooperative,
                                    (hipStream_t)stream, B->n_part, B->n_global_chunks, kl),
                  "batched persistent launch");
    }
    CS_BCHECK(launch_linear_add((int32_t)B->h.linA_idx.size(), B->d_linA_idx.p, B->d_linA_val.p, A,
                                (hipStream_t)stream), "linear-part launch");
    return CS_OK;
}

cs_status cs_batch_vjp(cs_batch *B, const double *x, double ag0, const double *hist,
                       const double *A_bar, const double *b_bar, double *W_bar, double *L_bar,
                       double *VTH0_bar, void *stream) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (!B->params_set) return bfail(CS_ESTATE, "cs_batch_set_params must come first");
    if (!x || !A_bar || !b_bar || !W_bar || !L_bar || !VTH0_bar) return bfail(CS_EINVAL, "NULL argument");
    if (cur_device() != B->device) return bfail(CS_ESTATE, "batch uploaded to another device");
    const KCirc kc = make_kc(B);
    const KCall call{x, ag0, hist, nullptr, nullptr};
    CS_BCHECK(launch_vjp(kc, call, A_bar, b_bar, W_bar, L_bar, VTH0_bar, (hipStream_t)stream), "vjp launch");
    return CS_OK;
}

cs_status cs_batch_set_schedule(cs_batch *B, cs_variant schedule) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (schedule != CS_COLOR_PERSISTENT && schedule != CS_COLOR_REGION)
        return bfail(CS_EINVAL, "batch schedule must be CS_COLOR_PERSISTENT or CS_COLOR_REGION");
    B->schedule = schedule;
    return CS_OK;
}

cs_status cs_batch_plan_regions(cs_batch *B, int32_t block) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (block < 64 || block > 256 || block % 64 != 0) return bfail(CS_EINVAL, "block must be 64, 128, 192 or 256");
    if (!B->packed) {
        try {
            cs_status st = pack(B);
            if (st != CS_OK) return st;
        } catch (const std::bad_alloc &) {
            return bfail(CS_ENOMEM, "host allocation");
        }
    }
    return plan_regions(B, block);
}

cs_status cs_batch_get_region_info(const cs_batch *B, int32_t *n_regions, int32_t *max_phases,
                                   int64_t *n_items, int64_t *n_staged, int64_t *n_interior,
                                   int64_t *n_links, int64_t *n_folds, int64_t *n_fold_src) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    region_info(B->rp, n_regions, max_phases, n_items, n_staged, n_interior, n_links, n_folds, n_fold_src);
    return CS_OK;
}

cs_status cs_batch_get_region_plan(const cs_batch *B, int32_t *perm, uint16_t *phase, int32_t *code,
                                   int32_t *rtab, int32_t *interior, int32_t *links, int32_t *item,
                                   int32_t *fold, int32_t *fold_src) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (!B->rp.built) return bfail(CS_ESTATE, "no region plan yet");
    region_tables(B->rp, perm, phase, code, rtab, interior, links, item, fold, fold_src);
    return CS_OK;
}

cs_status cs_batch_get_region_hubs(const cs_batch *B, int64_t *counts, int32_t *hfold, int32_t *part_ptr) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (!B->rp.built) return bfail(CS_ESTATE, "no region plan yet");
    region_hub_tables(B->rp, counts, hfold, part_ptr);
    return CS_OK;
}

cs_status cs_batch_check(cs_batch *B, void *stream) {
    if (!B) return bfail(CS_EINVAL, "NULL batch");
    if (B->device < 0) return CS_OK;
    CS_BCHECK(hipStreamSynchronize((hipStream_t)stream), "stream synchronise");
    uint32_t err = 0;
    CS_BCHECK(hipMemcpy(&err, B->d_sync.p + 1, sizeof(err), hipMemcpyDeviceToHost), "read error word");
    if (err) {
        CS_BCHECK(hipMemset(B->d_sync.p + 1, 0, sizeof(uint32_t)), "clear error word");
        if (B->d_hub_count.n)
            CS_BCHECK(hipMemset(B->d_hub_count.p, 0, sizeof(uint32_t) * B->d_hub_count.n), "clear hub counters");
        if (B->rd.item_count.n)
            CS_BCHECK(hipMemset(B->rd.item_count.p, 0, sizeof(uint32_t) * B->rd.item_count.n), "clear item counters");
        return bfail(CS_EDOMAIN, "a barrier wait exceeded its spin budget");
    }
    return CS_OK;
}

}  // extern "C"
