// C-ABI of the colorstamp library: argument and state checks, uploads, dispatch of
// the kernel variants.  No exception crosses the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "colorstamp.h"
#include "internal.hpp"
#include "launch.hpp"

namespace cs {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

KCirc make_kcirc(cs_circuit *c) {
    KCirc k{};
    const HostCircuit &h = c->h;
    k.n = h.n_dev;
    k.n_colors = h.n_colors;
    k.nc_max = h.max_nc;
    k.term = c->d_term.p;
    k.pol = c->d_pol.p;
    k.par = c->d_par.p;
    k.sdp = c->d_sdp.p;
    k.code = c->d_code.p;
    k.acode = c->d_acode.p;
    k.perm = c->d_perm.p;
    k.cptr = c->d_cptr.p;
    k.n_fixA = (int32_t)h.fixA_idx.size();
    k.n_fixB = (int32_t)h.fixB_idx.size();
    k.fixA_idx = c->d_fixA_idx.p;
    k.fixA_val = c->d_fixA_val.p;
    k.fixB_idx = c->d_fixB_idx.p;
    k.fixB_val = c->d_fixB_val.p;
    k.n_hub = (int32_t)h.hub_target.size();
    k.hub_ptr = c->d_hub_ptr.p;
    k.hub_target = c->d_hub_target.p;
    k.stage = c->d_stage.p;
    k.n_hub_chunks = (int32_t)h.hub_of_chunk.size();
    k.hub_cptr = c->d_hub_cptr.p;
    k.hub_of_chunk = c->d_hub_of_chunk.p;
    k.hub_part = c->d_hub_part.p;
    k.hub_count = c->d_hub_count.p;
    k.card[0] = c->card[0];
    k.card[1] = c->card[1];
    return k;
}

}  // namespace cs

using namespace cs;

namespace {

cs_status fail(cs_status st, const std::string &msg) {
    set_error(msg);
    return st;
}

cs_status hip_fail(hipError_t e, const char *what) {
    return fail(CS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define CS_CHECK_HIP(expr, what)                     \
    do {                                             \
        hipError_t e_ = (expr);                      \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

int current_device() {
    int d = -1;
    if (hipGetDevice(&d) != hipSuccess) return -1;
    return d;
}

// Order positions inside each colour by polarity (NMOS first), then device index,
// so that waves mostly hold one polarity.  Any order inside a colour is valid.
void order_within_colours(HostCircuit &h) {
    for (int32_t c = 0; c < h.n_colors; ++c) {
        auto b = h.perm.begin() + h.colour_ptr[(size_t)c];
        auto e = h.perm.begin() + h.colour_ptr[(size_t)c + 1];
        std::stable_sort(b, e, [&](int32_t x, int32_t y) {
            return (h.pol[(size_t)x] < 0) < (h.pol[(size_t)y] < 0);
        });
    }
}

// Colour-major SoA of the terminals: x index + 1 (0 = ground), offset by row_off.
std::vector<int32_t> colour_major_terms(const HostCircuit &h, int64_t row_off) {
    const size_t n = (size_t)h.n_dev;
    std::vector<int32_t> t(4 * n);
    for (size_t p = 0; p < n; ++p) {
        const int32_t v = h.perm[p];
        for (int j = 0; j < 4; ++j) {
            const int32_t nd = h.term[4 * (size_t)v + j];
            t[(size_t)j * n + p] = nd == 0 ? 0 : (int32_t)(row_off + nd);
        }
    }
    return t;
}

cs_status upload_circuit(cs_circuit *c) {
    HostCircuit &h = c->h;
    const size_t n = (size_t)h.n_dev;
    std::vector<int8_t> pol(n);
    for (size_t p = 0; p < n; ++p) pol[p] = h.pol[(size_t)h.perm[p]];
    CS_CHECK_HIP(c->d_term.upload(colour_major_terms(h, 0)), "upload terminals");
    CS_CHECK_HIP(c->d_pol.upload(pol), "upload polarity");
    CS_CHECK_HIP(c->d_code.upload(h.code), "upload stamp codes");
    CS_CHECK_HIP(c->d_acode.upload(h.acode), "upload atomic codes");
    CS_CHECK_HIP(c->d_perm.upload(h.perm), "upload permutation");
    c->d_ipos.release();   // rebuilt from the new positions at the next serial stamp
    CS_CHECK_HIP(c->d_cptr.upload(h.colour_ptr), "upload colour pointers");
    CS_CHECK_HIP(c->d_fixA_idx.upload(h.fixA_idx), "upload fixed stores");
    CS_CHECK_HIP(c->d_fixA_val.upload(h.fixA_val), "upload fixed stores");
    CS_CHECK_HIP(c->d_fixB_idx.upload(h.fixB_idx), "upload fixed stores");
    CS_CHECK_HIP(c->d_fixB_val.upload(h.fixB_val), "upload fixed stores");
    CS_CHECK_HIP(c->d_linA_idx.upload(h.linA_idx), "upload linear part");
    CS_CHECK_HIP(c->d_linA_val.upload(h.linA_val), "upload linear part");
    CS_CHECK_HIP(c->d_hub_ptr.upload(h.hub_ptr), "upload hub lists");
    CS_CHECK_HIP(c->d_hub_target.upload(h.hub_target), "upload hub lists");
    CS_CHECK_HIP(c->d_stage.alloc(h.hub_ptr.empty() ? 0 : (size_t)h.hub_ptr.back()), "alloc staging");
    CS_CHECK_HIP(c->d_hub_cptr.upload(h.hub_cptr), "upload hub chunks");
    CS_CHECK_HIP(c->d_hub_of_chunk.upload(h.hub_of_chunk), "upload hub chunks");
    CS_CHECK_HIP(c->d_hub_part.alloc(h.hub_of_chunk.size()), "alloc hub partials");
    CS_CHECK_HIP(c->d_hub_count.alloc(h.hub_target.size() * CNT_STRIDE), "alloc hub counters");
    if (!h.hub_target.empty())
        CS_CHECK_HIP(hipMemset(c->d_hub_count.p, 0, sizeof(uint32_t) * c->d_hub_count.n), "clear hub counters");
    CS_CHECK_HIP(c->d_par.alloc(3 * n), "alloc parameters");
    CS_CHECK_HIP(c->d_sdp.alloc((size_t)NSD * n), "alloc model constants");
    int dev_count = 0;
    CS_CHECK_HIP(hipGetDeviceCount(&dev_count), "device count");
    hipDeviceProp_t prop;
    CS_CHECK_HIP(hipGetDeviceProperties(&prop, current_device()), "device properties");
    const size_t words = 2 + (size_t)prop.multiProcessorCount * 64;
    CS_CHECK_HIP(c->d_sync.alloc(words), "alloc barrier state");
    CS_CHECK_HIP(hipMemset(c->d_sync.p, 0, words * sizeof(uint32_t)), "clear barrier state");
    c->device = current_device();
    c->grid = 0;
    c->params_set = false;
    return CS_OK;
}

// Grid of the persistent kernel for the current configuration.  phase_only: the
// evaluate-in-phase mode (the persistent variant's fallback when the regions cannot
// all be resident).
cs_status plan_persistent(cs_circuit *c, bool phase_only) {
    const int key = phase_only ? 1 : 2;
    if (c->grid > 0 && c->grid_key == key) return CS_OK;
    hipDeviceProp_t prop;
    CS_CHECK_HIP(hipGetDeviceProperties(&prop, c->device), "device properties");
    const int block = c->block;
    int per_cu_ahead = 0, per_cu_phase = 0;
    CS_CHECK_HIP(persistent_capacity(1, block, c->h.max_nc, &per_cu_ahead), "occupancy");
    CS_CHECK_HIP(persistent_capacity(0, block, c->h.max_nc, &per_cu_phase), "occupancy");
    const int64_t cap_ahead = (int64_t)per_cu_ahead * prop.multiProcessorCount;
    const int64_t cap_phase = (int64_t)per_cu_phase * prop.multiProcessorCount;
    const int64_t need_ahead = std::max<int64_t>(1, (c->h.n_dev + block - 1) / block);
    int64_t max_colour = 0;
    for (int32_t k = 0; k < c->h.n_colors; ++k)
        max_colour = std::max<int64_t>(max_colour, c->h.colour_ptr[k + 1] - c->h.colour_ptr[k]);
    const bool fits = !phase_only && need_ahead <= cap_ahead;
    if (!phase_only && c->eval_ahead_req == 1 && !fits)
        return fail(CS_ENOTSUP, "evaluate-ahead needs one resident thread per device");
    c->eval_ahead = c->eval_ahead_req == 0 ? 0 : (fits ? 1 : 0);
    int64_t grid = c->eval_ahead ? need_ahead
                                 : std::min<int64_t>(cap_phase, std::max<int64_t>(1, (max_colour + block - 1) / block));
    if (grid < 1 || cap_phase < 1) return fail(CS_ENOTSUP, "persistent kernel does not fit the device");
    if ((size_t)grid + 2 > c->d_sync.n) return fail(CS_ENOTSUP, "grid larger than the barrier state");
    c->grid = (int32_t)grid;
    c->grid_key = key;
    return CS_OK;
}

// Region planner input of a single circuit (colour-major table).
RegionSource region_source(const HostCircuit &h) {
    RegionSource src;
    src.n = h.n_dev;
    src.code = h.code;
    src.term = colour_major_terms(h, 0);
    src.pol.resize((size_t)h.n_dev);
    src.colour.resize((size_t)h.n_dev);
    for (size_t p = 0; p < (size_t)h.n_dev; ++p) {
        src.pol[p] = h.pol[(size_t)h.perm[p]];
        src.colour[p] = h.colour[(size_t)h.perm[p]];
    }
    src.perm = h.perm;
    src.nnz = h.nnz;
    src.n_rows = h.n_rows;
    src.hub_ptr = h.hub_ptr;
    src.hub_cptr = h.hub_cptr;
    src.stage_base = h.hub_ptr.empty() ? 0 : h.hub_ptr.back();
    return src;
}

// Compute units of the current GPU, 0 when there is none (host-only planning).
int32_t device_cus() {
    int dev = -1, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 0;
    (void)hipGetLastError();
    return cus;
}

cs_status plan_regions(cs_circuit *c, int32_t block) {
    const int32_t cus = c->plan_cus >= 0 ? c->plan_cus : device_cus();
    if (c->rp.built && c->rp.cap == block && c->rp.cus == cus) return CS_OK;
    c->rd.ready = false;
    try {
        RegionSource src = region_source(c->h);
        src.cus = cus;
        Err e = build_regions(src, block, c->rp);
        if (e.st == CS_OK && region_lds_bytes(c->rp.max_lds + 1, c->rp.max_nc, block) > (size_t)REGION_LDS_LIMIT)
            e = {CS_ENOTSUP, "region LDS exceeds 64 KiB; use a smaller block"};
        if (e.st != CS_OK) {
            c->rp = RegionPlan{};
            return fail(e.st, e.msg);
        }
    } catch (const std::bad_alloc &) {
        c->rp = RegionPlan{};
        return fail(CS_ENOMEM, "host allocation");
    }
    return CS_OK;
}

// Per-device model constants from the colour-major parameters and the cards (the
// kernels never see W, L, VTH0 themselves, except the adjoint), and their
// region-major copy when the region tables are on the device.  Launched on the
// caller's stream so that a captured step replayed after a parameter change reads
// the new values (a replay runs no host code); without uploaded region tables the
// copy is made when they are uploaded.
cs_status refresh_consts(cs_circuit *c, hipStream_t s) {
    CS_CHECK_HIP(launch_dev_const(make_kcirc(c), c->d_sdp.p, s), "model-constant launch");
    if (c->rd.ready) {
        CS_CHECK_HIP(launch_permute_rows(c->h.n_dev, c->rd.cm_pos.p, c->d_sdp.p, c->h.n_dev, NSD, c->rd.sdp.p, s),
                     "model-constant permute launch");
        c->rd.sdp_stale = false;
    } else {
        c->rd.sdp_stale = true;
    }
    return CS_OK;
}

// Region plan for the current block size, uploaded, and its parameter copy current.
cs_status ensure_region(cs_circuit *c, hipStream_t s) {
    cs_status st = plan_regions(c, c->block);
    if (st != CS_OK) return st;
    if (!c->rd.ready) {
        hipError_t e = upload_regions(c->rp, c->rd);
        if (e != hipSuccess) {
            c->rd.ready = false;
            return hip_fail(e, "upload region tables");
        }
    }
    if (c->rd.sdp_stale) {
        CS_CHECK_HIP(launch_permute_rows(c->h.n_dev, c->rd.cm_pos.p, c->d_sdp.p, c->h.n_dev, NSD, c->rd.sdp.p, s),
                     "model-constant permute launch");
        c->rd.sdp_stale = false;
    }
    return CS_OK;
}

}  // namespace

extern "C" {

const char *cs_last_error(void) { return g_err.c_str(); }

cs_status cs_circuit_create(int32_t n_nodes, int32_t n_dev, const int32_t *term, const int8_t *pol,
                            int32_t n_vsrc, const int32_t *vsrc, const double *vsrc_volts,
                            cs_circuit **out) {
    if (!out) return fail(CS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_nodes < 1 || n_dev < 0 || n_vsrc < 0) return fail(CS_EINVAL, "negative or empty sizes");
    if ((n_dev > 0 && (!term || !pol)) || (n_vsrc > 0 && (!vsrc || !vsrc_volts)))
        return fail(CS_EINVAL, "NULL input array");
    for (int64_t i = 0; i < 4 * (int64_t)n_dev; ++i)
        if (term[i] < 0 || term[i] >= n_nodes) return fail(CS_EINVAL, "terminal node id out of range");
    for (int32_t i = 0; i < n_dev; ++i)
        if (pol[i] != 1 && pol[i] != -1) return fail(CS_EINVAL, "polarity must be +1 or -1");
    for (int64_t i = 0; i < 2 * (int64_t)n_vsrc; ++i)
        if (vsrc[i] < 0 || vsrc[i] >= n_nodes) return fail(CS_EINVAL, "source node id out of range");
    if ((int64_t)n_dev * NCODE >= ((int64_t)1 << 31)) return fail(CS_ENOTSUP, "too many devices");
    cs_circuit *c = new (std::nothrow) cs_circuit();
    if (!c) return fail(CS_ENOMEM, "host allocation");
    try {
        c->h.n_nodes = n_nodes;
        c->h.n_dev = n_dev;
        c->h.n_vsrc = n_vsrc;
        c->h.term.assign(term, term + 4 * (size_t)n_dev);
        c->h.pol.assign(pol, pol + (size_t)n_dev);
        if (n_vsrc) {
            c->h.vsrc.assign(vsrc, vsrc + 2 * (size_t)n_vsrc);
            c->h.vsrc_volts.assign(vsrc_volts, vsrc_volts + (size_t)n_vsrc);
        }
    } catch (...) {
        delete c;
        return fail(CS_ENOMEM, "host allocation");
    }
    *out = c;
    return CS_OK;
}

void cs_circuit_destroy(cs_circuit *c) { delete c; }

cs_status cs_set_resistors(cs_circuit *c, int32_t n_res, const int32_t *nodes, const double *g) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (n_res < 0) return fail(CS_EINVAL, "negative resistor count");
    if (n_res > 0 && (!nodes || !g)) return fail(CS_EINVAL, "NULL input array");
    if (c->h.mapped) return fail(CS_ESTATE, "resistors must be set before cs_build_stamp_map");
    if (2 * (int64_t)n_res >= INDEX_LIMIT) return fail(CS_ENOTSUP, "too many resistors");
    for (int64_t i = 0; i < 2 * (int64_t)n_res; ++i)
        if (nodes[i] < 0 || nodes[i] >= c->h.n_nodes) return fail(CS_EINVAL, "resistor node id out of range");
    for (int32_t i = 0; i < n_res; ++i)
        if (!std::isfinite(g[i])) return fail(CS_EINVAL, "resistor conductance not finite");
    try {
        c->h.res.assign(nodes, nodes + 2 * (size_t)n_res);
        c->h.res_g.assign(g, g + (size_t)n_res);
    } catch (...) {
        return fail(CS_ENOMEM, "host allocation");
    }
    return CS_OK;
}

cs_status cs_build_coloring(cs_circuit *c, const uint8_t *exclude, int32_t *n_colors,
                            int32_t *colour_out, int64_t *n_edges) {
    return cs_build_coloring_order(c, exclude, CS_ORDER_NATURAL, n_colors, colour_out, n_edges);
}

cs_status cs_build_coloring_order(cs_circuit *c, const uint8_t *exclude, int32_t order, int32_t *n_colors,
                                  int32_t *colour_out, int64_t *n_edges) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    try {
        Err e = build_colouring(c->h, exclude, n_edges, order);
        if (e.st != CS_OK) return fail(e.st, e.msg);
        order_within_colours(c->h);
        c->rp = RegionPlan{};
        c->rd.ready = false;
    } catch (const std::bad_alloc &) {
        return fail(CS_ENOMEM, "host allocation");
    }
    c->grid = 0;
    c->device = -1;
    if (n_colors) *n_colors = c->h.n_colors;
    if (colour_out) std::memcpy(colour_out, c->h.colour.data(), sizeof(int32_t) * c->h.n_dev);
    return CS_OK;
}

cs_status cs_build_stamp_map(cs_circuit *c, int32_t *n_rows, int64_t *nnz) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->h.coloured) return fail(CS_ESTATE, "cs_build_coloring must come first");
    try {
        destroy_newton(c->newton);   // the solver's factor pattern belongs to the old map
        c->newton = nullptr;
        Err e = build_map(c->h);
        c->rp = RegionPlan{};
        c->rd.ready = false;
        if (e.st != CS_OK) return fail(e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(CS_ENOMEM, "host allocation");
    }
    c->device = -1;
    c->grid = 0;
    if (n_rows) *n_rows = c->h.n_rows;
    if (nnz) *nnz = c->h.nnz;
    return CS_OK;
}

cs_status cs_get_pattern(const cs_circuit *c, int32_t *row_ptr, int32_t *col_idx) {
    if (!c || !row_ptr || !col_idx) return fail(CS_EINVAL, "NULL argument");
    if (!c->h.mapped) return fail(CS_ESTATE, "cs_build_stamp_map must come first");
    std::memcpy(row_ptr, c->h.row_ptr.data(), sizeof(int32_t) * c->h.row_ptr.size());
    std::memcpy(col_idx, c->h.col_idx.data(), sizeof(int32_t) * c->h.col_idx.size());
    return CS_OK;
}

cs_status cs_get_stamp_map(const cs_circuit *c, int32_t *slot, int8_t *sflag, int32_t *brow,
                           int8_t *bflag) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    const HostCircuit &h = c->h;
    if (!h.mapped) return fail(CS_ESTATE, "cs_build_stamp_map must come first");
    const size_t n = (size_t)h.n_dev;
    for (size_t p = 0; p < n; ++p) {
        const size_t v = (size_t)h.perm[p];
        int32_t u[4];
        int k = 0;
        for (int t = 0; t < 4; ++t) {
            const int32_t nd = h.term[4 * v + t];
            if (nd == 0) continue;
            bool seen = false;
            for (int j = 0; j < k; ++j) seen = seen || u[j] == nd;
            if (!seen) u[k++] = nd;
        }
        for (int j = 0; j < 16; ++j) {
            if (slot) slot[16 * v + j] = -1;
            if (sflag) sflag[16 * v + j] = -1;
        }
        for (int j = 0; j < 4; ++j) {
            if (brow) brow[4 * v + j] = -1;
            if (bflag) bflag[4 * v + j] = -1;
        }
        for (int j = 0; j < k * k + k; ++j) {
            const uint32_t cd = (uint32_t)h.code[(size_t)j * n + p];
            const int8_t tag = (int8_t)(cd >> 30);
            const int32_t target = h.acode[(size_t)j * n + p];
            if (j < k * k) {
                if (slot) slot[16 * v + j] = target;
                if (sflag) sflag[16 * v + j] = tag;
            } else {
                if (brow) brow[4 * v + (j - k * k)] = target;
                if (bflag) bflag[4 * v + (j - k * k)] = tag;
            }
        }
    }
    return CS_OK;
}

cs_status cs_set_models(cs_circuit *c, const cs_model_card *nmos, const cs_model_card *pmos) {
    if (!c || !nmos || !pmos) return fail(CS_EINVAL, "NULL argument");
    if (nmos->size != sizeof(cs_model_card) || pmos->size != sizeof(cs_model_card))
        return fail(CS_EINVAL, "model card size mismatch");
    for (const cs_model_card *m : {nmos, pmos}) {
        if (m->jmod == 0.0) continue;
        const double vt = 8.617333262e-5 * m->tnom;
        if (!(m->nj > 0.0) || !(m->pb > 0.0) || !(m->fc >= 0.0 && m->fc < 1.0) || !(m->js >= 0.0) ||
            !(m->cj >= 0.0) || !(m->hdif >= 0.0) || !(m->vjmax <= 40.0 * (m->nj * vt)))
            return fail(CS_EINVAL, "junction parameters out of range");
    }
    c->card[0] = derive_card(*nmos);
    c->card[1] = derive_card(*pmos);
    c->models_set = true;
    // the per-device constants depend on the cards: recompute them from the set
    // parameters (null stream), or ask for the parameters again on another device
    if (c->params_set) {
        if (current_device() != c->device) {
            c->params_set = false;
            return CS_OK;
        }
        return refresh_consts(c, nullptr);
    }
    return CS_OK;
}

cs_status cs_set_params(cs_circuit *c, const double *W, const double *L, const double *VTH0,
                        void *stream) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return fail(CS_ESTATE, "cs_build_stamp_map must come first");
    if (c->device < 0) {
        cs_status st = upload_circuit(c);
        if (st != CS_OK) return st;
    }
    if (c->h.n_dev > 0 && (!W || !L || !VTH0)) return fail(CS_EINVAL, "NULL parameter array");
    if (current_device() != c->device) return fail(CS_ESTATE, "circuit uploaded to another device");
    CS_CHECK_HIP(launch_gather_params(c->h.n_dev, c->d_perm.p, W, L, VTH0, c->d_par.p,
                                      (hipStream_t)stream), "parameter gather launch");
    c->params_set = true;
    return refresh_consts(c, (hipStream_t)stream);
}

cs_status cs_set_launch(cs_circuit *c, int32_t block, int32_t eval_ahead, int32_t cooperative) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (cooperative != 0 && cooperative != 1) return fail(CS_EINVAL, "cooperative must be 0 or 1");
    c->cooperative = cooperative == 1;
    if (block != 0 && (block < 64 || block > 256 || block % 64 != 0))
        return fail(CS_EINVAL, "block must be 64, 128, 192 or 256");
    if (eval_ahead < -1 || eval_ahead > 1) return fail(CS_EINVAL, "eval_ahead must be -1, 0 or 1");
    c->block = block ? block : 256;
    c->eval_ahead_req = eval_ahead;
    c->grid = 0;
    return CS_OK;
}

cs_status cs_set_plan_units(cs_circuit *c, int32_t cus) {
    if (!c || cus < -1) return fail(CS_EINVAL, "bad argument");
    c->plan_cus = cus;
    return CS_OK;
}

cs_status cs_set_spin_limit(cs_circuit *c, int64_t spins) {
    if (!c || spins < 0) return fail(CS_EINVAL, "bad argument");
    c->spin_limit = spins ? spins : (1 << 22);
    return CS_OK;
}

cs_status cs_get_info(const cs_circuit *c, int64_t *n_dev, int32_t *n_rows, int64_t *nnz,
                      int32_t *n_colors, int32_t *grid, int32_t *block, int32_t *eval_ahead,
                      int32_t *n_hub) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (n_dev) *n_dev = c->h.n_dev;
    if (n_rows) *n_rows = c->h.n_rows;
    if (nnz) *nnz = c->h.nnz;
    if (n_colors) *n_colors = c->h.n_colors;
    if (grid) *grid = c->grid;
    if (block) *block = c->block;
    if (eval_ahead) *eval_ahead = c->eval_ahead;
    if (n_hub) *n_hub = (int32_t)c->h.hub_target.size();
    return CS_OK;
}

// The device contributions under one schedule (everything but the linear part).
static cs_status eval_devices(cs_circuit *c, cs_variant variant, const KCall &call, hipStream_t s) {
    const KCirc kc = make_kcirc(c);
    switch (variant) {
        case CS_COLOR_PERSISTENT:
            if (c->eval_ahead_req != 0) {
                // every region resident at once: the grid-barrier form of the region
                // schedule (workgroup colour phases in LDS, shared entries in place)
                cs_status st = ensure_region(c, s);
                if (st != CS_OK) return st;
                if (c->rg_cap_block != c->block || c->rg_cap_regions != c->rp.n_regions) {
                    int per_cu = 0;
                    CS_CHECK_HIP(region_grid_capacity(c->block, (c->rp.max_lds + 1) & ~1, c->rp.max_nc, &per_cu),
                                 "occupancy");
                    hipDeviceProp_t prop;
                    CS_CHECK_HIP(hipGetDeviceProperties(&prop, c->device), "device properties");
                    c->rg_cap = (int64_t)per_cu * prop.multiProcessorCount;
                    c->rg_cap_block = c->block;
                    c->rg_cap_regions = c->rp.n_regions;
                }
                const int64_t cap = c->rg_cap;
                const int32_t nr = c->rp.n_regions;
                if (nr >= 1 && nr <= cap && (size_t)nr + 2 <= c->d_sync.n && c->rp.max_glevel >= 0) {
                    const KSync ks{c->d_sync.p, c->spin_limit};
                    CS_CHECK_HIP(launch_region_grid(region_kcirc(kc, c->rp, c->rd), call, region_kregion(c->rp, c->rd),
                                                    ks, c->block, c->cooperative, s), "persistent launch");
                    c->grid = nr;
                    c->grid_key = 3;
                    c->eval_ahead = 1;
                    return CS_OK;
                }
                if (c->eval_ahead_req == 1 && nr >= 1)
                    return fail(CS_ENOTSUP, "evaluate-ahead needs every region resident at once");
            }
            [[fallthrough]];
        case CS_COLOR_BUFFERED: {
            cs_status st = plan_persistent(c, variant == CS_COLOR_PERSISTENT);
            if (st != CS_OK) return st;
            int mode = c->eval_ahead;
            int grid = c->grid;
            if (variant == CS_COLOR_BUFFERED) {
                if (c->d_buf.n < (size_t)NCODE * c->h.n_dev)
                    CS_CHECK_HIP(c->d_buf.alloc((size_t)NCODE * c->h.n_dev), "alloc buffer");
                CS_CHECK_HIP(launch_eval_buffer(kc, call, c->d_buf.p, s), "evaluate launch");
                mode = 2;
                if (c->eval_ahead) {
                    // the stamp-only grid only needs the largest colour
                    int64_t mc = 0;
                    for (int32_t k = 0; k < c->h.n_colors; ++k)
                        mc = std::max<int64_t>(mc, c->h.colour_ptr[k + 1] - c->h.colour_ptr[k]);
                    grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, (mc + c->block - 1) / c->block));
                }
            }
            const KSync ks{c->d_sync.p, c->spin_limit};
            const KLocal none{0, nullptr, nullptr};
            CS_CHECK_HIP(launch_persistent(kc, call, ks, c->d_buf.p, mode, grid, c->block,
                                           c->cooperative, s, grid, kc.n_hub_chunks, none),
                         "persistent launch");
            return CS_OK;
        }
        case CS_COLOR_PER_KERNEL: {
            const HostCircuit &h = c->h;
            if (h.n_colors == 0) CS_CHECK_HIP(launch_fixed(kc, call, s), "fixed-store launch");
            for (int32_t k = 0; k < h.n_colors; ++k)
                CS_CHECK_HIP(launch_colour_phase(kc, call, k, h.colour_ptr[k + 1] - h.colour_ptr[k],
                                                 k == 0, s), "colour launch");
            CS_CHECK_HIP(launch_hub(kc, call, s), "hub launch");
            return CS_OK;
        }
        case CS_ATOMIC:
            CS_CHECK_HIP(launch_atomic(kc, call, c->h.nnz, c->h.n_rows, s), "atomic launch");
            return CS_OK;
        case CS_ATOMIC_WAVE:
            CS_CHECK_HIP(launch_atomic_wave(kc, call, c->h.nnz, c->h.n_rows, s), "atomic launch");
            return CS_OK;
        case CS_SERIAL_STAMP: {
            const HostCircuit &h = c->h;
            if (c->d_buf.n < (size_t)NCODE * h.n_dev)
                CS_CHECK_HIP(c->d_buf.alloc((size_t)NCODE * h.n_dev), "alloc buffer");
            if (c->d_ipos.n != (size_t)h.n_dev) {
                std::vector<int32_t> ipos((size_t)h.n_dev);
                for (int32_t p = 0; p < h.n_dev; ++p) ipos[(size_t)h.perm[(size_t)p]] = p;
                CS_CHECK_HIP(c->d_ipos.upload(ipos), "upload positions");
            }
            CS_CHECK_HIP(launch_serial(kc, call, h.nnz, h.n_rows, c->d_buf.p, c->d_ipos.p, s), "serial launch");
            return CS_OK;
        }
        case CS_COLOR_REGION: {
            cs_status st = ensure_region(c, s);
            if (st != CS_OK) return st;
            CS_CHECK_HIP(launch_region(region_kcirc(kc, c->rp, c->rd), call, region_kregion(c->rp, c->rd),
                                       c->block, s), "region launch");
            return CS_OK;
        }
        default:
            return fail(CS_EINVAL, "unknown variant");
    }
}

cs_status cs_eval_stamp(cs_circuit *c, cs_variant variant, const double *x, double ag0,
                        const double *hist, double *A_val, double *b, void *stream) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return fail(CS_ESTATE, "cs_build_stamp_map must come first");
    if (!c->models_set) return fail(CS_ESTATE, "cs_set_models must come first");
    if (!c->params_set) return fail(CS_ESTATE, "cs_set_params must come first");
    if (!x || !A_val || !b) return fail(CS_EINVAL, "NULL x, A or b");
    if (current_device() != c->device) return fail(CS_ESTATE, "circuit uploaded to another device");
    hipStream_t s = (hipStream_t)stream;
    const KCall call{x, ag0, hist, A_val, b};
    cs_status st = eval_devices(c, variant, call, s);
    if (st != CS_OK) return st;
    // series resistors on entries that devices also write: added after every contribution
    CS_CHECK_HIP(launch_linear_add((int32_t)c->h.linA_idx.size(), c->d_linA_idx.p, c->d_linA_val.p, A_val, s),
                 "linear-part launch");
    return CS_OK;
}

cs_status cs_history(cs_circuit *c, const double *x, double ag0, double *hist_out, void *stream) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return fail(CS_ESTATE, "cs_build_stamp_map must come first");
    if (!c->models_set) return fail(CS_ESTATE, "cs_set_models must come first");
    if (!c->params_set) return fail(CS_ESTATE, "cs_set_params must come first");
    if (!x || !hist_out) return fail(CS_EINVAL, "NULL x or hist_out");
    if (current_device() != c->device) return fail(CS_ESTATE, "circuit uploaded to another device");
    const KCall call{x, ag0, nullptr, nullptr, nullptr};
    CS_CHECK_HIP(launch_history(make_kcirc(c), call, hist_out, (hipStream_t)stream), "history launch");
    return CS_OK;
}

cs_status cs_plan_regions(cs_circuit *c, int32_t block) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->h.mapped) return fail(CS_ESTATE, "cs_build_stamp_map must come first");
    if (block < 64 || block > 256 || block % 64 != 0) return fail(CS_EINVAL, "block must be 64, 128, 192 or 256");
    return plan_regions(c, block);
}

cs_status cs_get_region_info(const cs_circuit *c, int32_t *n_regions, int32_t *max_phases,
                             int64_t *n_items, int64_t *n_staged, int64_t *n_interior, int64_t *n_links,
                             int64_t *n_folds, int64_t *n_fold_src) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    region_info(c->rp, n_regions, max_phases, n_items, n_staged, n_interior, n_links, n_folds, n_fold_src);
    return CS_OK;
}

cs_status cs_get_region_plan(const cs_circuit *c, int32_t *perm, uint16_t *phase, int32_t *code,
                             int32_t *rtab, int32_t *interior, int32_t *links, int32_t *item, int32_t *fold,
                             int32_t *fold_src) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->rp.built) return fail(CS_ESTATE, "no region plan yet");
    region_tables(c->rp, perm, phase, code, rtab, interior, links, item, fold, fold_src);
    return CS_OK;
}

cs_status cs_get_region_hubs(const cs_circuit *c, int64_t *counts, int32_t *hfold, int32_t *part_ptr) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (!c->rp.built) return fail(CS_ESTATE, "no region plan yet");
    region_hub_tables(c->rp, counts, hfold, part_ptr);
    return CS_OK;
}

cs_status cs_check(cs_circuit *c, void *stream) {
    if (!c) return fail(CS_EINVAL, "NULL circuit");
    if (c->device < 0) return CS_OK;
    CS_CHECK_HIP(hipStreamSynchronize((hipStream_t)stream), "stream synchronise");
    uint32_t err = 0;
    CS_CHECK_HIP(hipMemcpy(&err, c->d_sync.p + 1, sizeof(err), hipMemcpyDeviceToHost), "read error word");
    if (err) {
        CS_CHECK_HIP(hipMemset(c->d_sync.p + 1, 0, sizeof(uint32_t)), "clear error word");
        if (c->d_hub_count.n)
            CS_CHECK_HIP(hipMemset(c->d_hub_count.p, 0, sizeof(uint32_t) * c->d_hub_count.n), "clear hub counters");
        // the grid-barrier form of the region schedule counts in the region tables
        if (c->rd.item_count.n)
            CS_CHECK_HIP(hipMemset(c->rd.item_count.p, 0, sizeof(uint32_t) * c->rd.item_count.n), "clear item counters");
        return fail(CS_EDOMAIN, "a barrier wait exceeded its spin budget");
    }
    return CS_OK;
}

}  // extern "C"
