// Host setup: conflict graph, greedy colouring, CSR pattern, stamp map, hub lists.
//
// Paper, Methodology: the FET conflict graph is built at circuit setup, one vertex
// per FET and an edge between FETs sharing a non-ground node; the greedy colouring
// (Introduction) visits vertices in order and gives each the smallest colour not
// used by an already coloured neighbour.  The graph stays implicit here: a colour
// is forbidden for a device exactly when it is already used on one of the
// device's conflict nodes, so each node keeps a bitset of its used colours.  Besides
// the paper's ascending order, the vertices can be visited largest degree first
// (Welsh and Powell) or by DSATUR (Brelaz), which often reach the clique bound.
#include <algorithm>
#include <cstring>
#include <set>
#include <tuple>
#include <cmath>
#include <unordered_map>

#include "internal.hpp"

namespace cs {

namespace {

// Distinct non-ground nodes of a device in first-appearance order over (d, g, s, b).
int unique_nodes(const int32_t *t4, int32_t u[4]) {
    int k = 0;
    for (int t = 0; t < 4; ++t) {
        if (t4[t] == 0) continue;
        bool seen = false;
        for (int j = 0; j < k; ++j) seen = seen || (u[j] == t4[t]);
        if (!seen) u[k++] = t4[t];
    }
    return k;
}

// Number of unordered device pairs sharing at least one conflict node, by
// inclusion-exclusion over the node subsets each device touches:
// sum over nonempty subsets U of (-1)^(|U|+1) * C(devices containing U, 2).
struct SubsetKey {
    int32_t n[4];
    bool operator==(const SubsetKey &o) const {
        return n[0] == o.n[0] && n[1] == o.n[1] && n[2] == o.n[2] && n[3] == o.n[3];
    }
};
struct SubsetHash {
    size_t operator()(const SubsetKey &k) const {
        uint64_t h = 1469598103934665603ull;
        for (int i = 0; i < 4; ++i) h = (h ^ (uint64_t)(uint32_t)k.n[i]) * 1099511628211ull;
        return (size_t)h;
    }
};

int64_t count_edges(const HostCircuit &h) {
    std::unordered_map<SubsetKey, int64_t, SubsetHash> cnt;
    cnt.reserve((size_t)h.n_dev * 4);
    for (int32_t v = 0; v < h.n_dev; ++v) {
        int32_t u[4];
        int k = unique_nodes(&h.term[4 * (size_t)v], u);
        int32_t c[4];
        int m = 0;
        for (int j = 0; j < k; ++j)
            if (!h.excl[u[j]]) c[m++] = u[j];
        std::sort(c, c + m);
        for (int mask = 1; mask < (1 << m); ++mask) {
            SubsetKey key{{-1, -1, -1, -1}};
            int w = 0;
            for (int j = 0; j < m; ++j)
                if (mask & (1 << j)) key.n[w++] = c[j];
            cnt[key]++;
        }
    }
    int64_t e = 0;
    for (auto &kv : cnt) {
        int sz = 0;
        while (sz < 4 && kv.first.n[sz] >= 0) ++sz;
        const int64_t pairs = kv.second * (kv.second - 1) / 2;
        e += (sz % 2 == 1) ? pairs : -pairs;
    }
    return e;
}

}  // namespace

Err build_colouring(HostCircuit &h, const uint8_t *exclude, int64_t *n_edges, int order) {
    if (order < 0 || order > 2) return {CS_EINVAL, "unknown colouring order"};
    h.excl.assign((size_t)h.n_nodes, 0);
    if (exclude)
        for (int32_t n = 0; n < h.n_nodes; ++n) h.excl[n] = exclude[n] ? 1 : 0;
    h.excl[0] = 1;  // ground never conflicts
    const size_t n = (size_t)h.n_dev;
    // conflict nodes of each device (distinct, non-excluded)
    std::vector<int32_t> cn(4 * n, -1);
    std::vector<int8_t> ncn(n, 0);
    for (size_t v = 0; v < n; ++v) {
        int32_t u[4];
        const int k = unique_nodes(&h.term[4 * v], u);
        for (int j = 0; j < k; ++j)
            if (!h.excl[u[j]]) cn[4 * v + (size_t)ncn[v]++] = u[j];
    }
    std::vector<std::vector<uint64_t>> used((size_t)h.n_nodes);
    auto smallest_free = [&](size_t v, std::vector<uint64_t> &acc) {
        size_t words = 0;
        for (int j = 0; j < ncn[v]; ++j) words = std::max(words, used[(size_t)cn[4 * v + j]].size());
        acc.assign(words + 1, 0);
        for (int j = 0; j < ncn[v]; ++j) {
            const auto &bs = used[(size_t)cn[4 * v + j]];
            for (size_t w = 0; w < bs.size(); ++w) acc[w] |= bs[w];
        }
        size_t w = 0;
        while (acc[w] == ~0ull) ++w;
        return (int32_t)(w * 64 + __builtin_ctzll(~acc[w]));
    };
    auto node_has = [&](int32_t node, int32_t c) {
        const auto &bs = used[(size_t)node];
        return (size_t)(c / 64) < bs.size() && ((bs[(size_t)(c / 64)] >> (c % 64)) & 1ull);
    };
    auto mark = [&](int32_t node, int32_t c) {
        auto &bs = used[(size_t)node];
        if (bs.size() <= (size_t)(c / 64)) bs.resize((size_t)(c / 64) + 1, 0);
        bs[(size_t)(c / 64)] |= 1ull << (c % 64);
    };
    h.colour.assign(n, -1);
    int32_t C = 0;
    std::vector<uint64_t> acc;
    if (order == 0) {
        // the paper's order: ascending device index
        for (size_t v = 0; v < n; ++v) {
            const int32_t c = smallest_free(v, acc);
            h.colour[v] = c;
            C = std::max(C, c + 1);
            for (int j = 0; j < ncn[v]; ++j) mark(cn[4 * v + j], c);
        }
    } else {
        // devices on each conflict node, and each device's degree (distinct neighbours)
        std::vector<int64_t> nptr((size_t)h.n_nodes + 1, 0);
        for (size_t v = 0; v < n; ++v)
            for (int j = 0; j < ncn[v]; ++j) nptr[(size_t)cn[4 * v + j] + 1]++;
        for (int32_t x = 0; x < h.n_nodes; ++x) nptr[(size_t)x + 1] += nptr[(size_t)x];
        std::vector<int32_t> on((size_t)nptr[(size_t)h.n_nodes]);
        {
            std::vector<int64_t> f(nptr.begin(), nptr.end() - 1);
            for (size_t v = 0; v < n; ++v)
                for (int j = 0; j < ncn[v]; ++j) on[(size_t)f[(size_t)cn[4 * v + j]]++] = (int32_t)v;
        }
        std::vector<int64_t> deg(n, 0);
        {
            std::vector<int32_t> seen(n, -1);
            for (size_t v = 0; v < n; ++v)
                for (int j = 0; j < ncn[v]; ++j) {
                    const int32_t x = cn[4 * v + j];
                    for (int64_t e = nptr[(size_t)x]; e < nptr[(size_t)x + 1]; ++e) {
                        const int32_t w = on[(size_t)e];
                        if ((size_t)w == v || seen[(size_t)w] == (int32_t)v) continue;
                        seen[(size_t)w] = (int32_t)v;
                        ++deg[v];
                    }
                }
        }
        if (order == 1) {
            // largest degree first, ties by ascending index
            std::vector<int32_t> seq(n);
            for (size_t v = 0; v < n; ++v) seq[v] = (int32_t)v;
            std::stable_sort(seq.begin(), seq.end(), [&](int32_t a, int32_t b) { return deg[(size_t)a] > deg[(size_t)b]; });
            for (int32_t vv : seq) {
                const size_t v = (size_t)vv;
                const int32_t c = smallest_free(v, acc);
                h.colour[v] = c;
                C = std::max(C, c + 1);
                for (int j = 0; j < ncn[v]; ++j) mark(cn[4 * v + j], c);
            }
        } else {
            // DSATUR: most distinct neighbour colours first, then larger degree, then
            // smaller index; a neighbour's saturation grows when a colour first
            // appears on one of its conflict nodes
            std::vector<int32_t> sat(n, 0);
            auto key = [&](size_t v) { return std::make_tuple(-(int64_t)sat[v], -deg[v], (int64_t)v); };
            std::set<std::tuple<int64_t, int64_t, int64_t>> open;
            for (size_t v = 0; v < n; ++v) open.insert(key(v));
            while (!open.empty()) {
                const size_t v = (size_t)std::get<2>(*open.begin());
                open.erase(open.begin());
                const int32_t c = smallest_free(v, acc);
                h.colour[v] = c;
                C = std::max(C, c + 1);
                for (int j = 0; j < ncn[v]; ++j) {
                    const int32_t x = cn[4 * v + j];
                    for (int64_t e = nptr[(size_t)x]; e < nptr[(size_t)x + 1]; ++e) {
                        const size_t u = (size_t)on[(size_t)e];
                        if (u == v || h.colour[u] >= 0) continue;
                        bool present = false;
                        for (int i2 = 0; i2 < ncn[u] && !present; ++i2) present = node_has(cn[4 * u + i2], c);
                        if (present) continue;
                        open.erase(key(u));
                        ++sat[u];
                        open.insert(key(u));
                    }
                    mark(x, c);
                }
            }
        }
    }
    h.n_colors = C;
    // colour-major order, stable in device index
    h.colour_ptr.assign((size_t)C + 1, 0);
    for (int32_t v = 0; v < h.n_dev; ++v) h.colour_ptr[(size_t)h.colour[v] + 1]++;
    for (int32_t c = 0; c < C; ++c) h.colour_ptr[c + 1] += h.colour_ptr[c];
    std::vector<int32_t> fill(h.colour_ptr.begin(), h.colour_ptr.end() - 1);
    h.perm.assign((size_t)h.n_dev, 0);
    for (int32_t v = 0; v < h.n_dev; ++v) h.perm[(size_t)fill[h.colour[v]]++] = v;
    if (n_edges) *n_edges = count_edges(h);
    h.coloured = true;
    h.mapped = false;
    return {CS_OK, ""};
}

Err build_map(HostCircuit &h) {
    const int32_t n_node_rows = h.n_nodes - 1;
    const int64_t n_rows = (int64_t)n_node_rows + h.n_vsrc;
    if (n_rows >= INDEX_LIMIT) return {CS_ENOTSUP, "too many MNA rows for 30-bit stamp codes"};
    h.n_rows = (int32_t)n_rows;

    // pattern: per row, the set of columns
    std::vector<std::vector<int32_t>> cols((size_t)n_rows);
    for (int32_t r = 0; r < n_node_rows; ++r) cols[(size_t)r].push_back(r);
    for (int32_t v = 0; v < h.n_dev; ++v) {
        int32_t u[4];
        int k = unique_nodes(&h.term[4 * (size_t)v], u);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b) cols[(size_t)u[a] - 1].push_back(u[b] - 1);
    }
    for (int32_t j = 0; j < h.n_vsrc; ++j) {
        int32_t br = n_node_rows + j;
        for (int e = 0; e < 2; ++e) {
            int32_t nd = h.vsrc[2 * (size_t)j + e];
            if (nd == 0) continue;
            cols[(size_t)nd - 1].push_back(br);
            cols[(size_t)br].push_back(nd - 1);
        }
    }
    const size_t n_res = h.res_g.size();
    for (size_t j = 0; j < n_res; ++j) {
        const int32_t p = h.res[2 * j], q = h.res[2 * j + 1];
        if (p == 0 || q == 0) continue;
        cols[(size_t)p - 1].push_back(q - 1);
        cols[(size_t)q - 1].push_back(p - 1);
    }
    h.row_ptr.assign((size_t)n_rows + 1, 0);
    h.col_idx.clear();
    for (int64_t r = 0; r < n_rows; ++r) {
        auto &c = cols[(size_t)r];
        std::sort(c.begin(), c.end());
        c.erase(std::unique(c.begin(), c.end()), c.end());
        h.col_idx.insert(h.col_idx.end(), c.begin(), c.end());
        h.row_ptr[(size_t)r + 1] = (int32_t)h.col_idx.size();
        if ((int64_t)h.col_idx.size() >= INDEX_LIMIT)
            return {CS_ENOTSUP, "too many nonzeros for 30-bit stamp codes"};
        std::vector<int32_t>().swap(c);
    }
    h.nnz = (int64_t)h.col_idx.size();
    auto slot_of = [&](int32_t r, int32_t c) -> int32_t {
        auto b = h.col_idx.begin() + h.row_ptr[(size_t)r];
        auto e = h.col_idx.begin() + h.row_ptr[(size_t)r + 1];
        auto it = std::lower_bound(b, e, c);
        return (it != e && *it == c) ? (int32_t)(it - h.col_idx.begin()) : -1;
    };

    // stamp codes in colour-major order; first encounter of an entry = first writer
    const size_t n = (size_t)h.n_dev;
    h.code.assign((size_t)NCODE * n, 0);
    h.acode.assign((size_t)NCODE * n, 0);
    std::vector<int32_t> wrote_A((size_t)h.nnz, -1), wrote_b((size_t)n_rows, -1);
    h.max_nc = 0;
    struct HubRef { int64_t target; int32_t dev; int32_t pos; int32_t j; };
    std::vector<HubRef> hubs;
    for (size_t p = 0; p < n; ++p) {
        const int32_t v = h.perm[p];
        const int32_t col = h.colour[(size_t)v];
        int32_t u[4];
        int k = unique_nodes(&h.term[4 * (size_t)v], u);
        h.max_nc = std::max(h.max_nc, k * k + k);
        for (int a = 0; a < k; ++a) {
            for (int b = 0; b < k; ++b) {
                const int j = a * k + b;
                int32_t s = slot_of(u[a] - 1, u[b] - 1);
                h.acode[(size_t)j * n + p] = s;
                if (h.excl[u[a]] && h.excl[u[b]]) {
                    hubs.push_back({s, v, (int32_t)p, j});
                    continue;
                }
                uint32_t tag = TAG_ADD;
                if (wrote_A[(size_t)s] < 0) tag = TAG_STORE;
                else if (wrote_A[(size_t)s] == col)
                    return {CS_EINVAL, "two devices of one colour share a matrix entry"};
                wrote_A[(size_t)s] = col;
                h.code[(size_t)j * n + p] = (int32_t)((tag << 30) | (uint32_t)s);
            }
            const int j = k * k + a;
            const int32_t r = u[a] - 1;
            h.acode[(size_t)j * n + p] = r;
            if (h.excl[u[a]]) {
                hubs.push_back({h.nnz + r, v, (int32_t)p, j});
                continue;
            }
            uint32_t tag = TAG_ADD;
            if (wrote_b[(size_t)r] < 0) tag = TAG_STORE;
            else if (wrote_b[(size_t)r] == col)
                return {CS_EINVAL, "two devices of one colour share a RHS row"};
            wrote_b[(size_t)r] = col;
            h.code[(size_t)j * n + p] = (int32_t)((tag << 30) | (uint32_t)r);
        }
    }
    // hub outputs: contributions staged in ascending device index per output
    std::sort(hubs.begin(), hubs.end(), [](const HubRef &x, const HubRef &y) {
        return x.target != y.target ? x.target < y.target : x.dev < y.dev;
    });
    if ((int64_t)hubs.size() >= INDEX_LIMIT) return {CS_ENOTSUP, "too many hub contributions"};
    h.hub_ptr.assign(1, 0);
    h.hub_target.clear();
    h.max_hub_len = 0;
    for (size_t i = 0; i < hubs.size(); ++i) {
        if (i == 0 || hubs[i].target != hubs[i - 1].target) {
            if (i > 0) h.hub_ptr.push_back((int32_t)i);
            const int64_t t = hubs[i].target;
            h.hub_target.push_back(t < h.nnz ? (int32_t)t
                                             : (int32_t)((uint32_t)(t - h.nnz) | HUB_B_FLAG));
            if (t < h.nnz) wrote_A[(size_t)t] = 0; else wrote_b[(size_t)(t - h.nnz)] = 0;
        }
        h.code[(size_t)hubs[i].j * n + (size_t)hubs[i].pos] =
            (int32_t)((TAG_HUB << 30) | (uint32_t)i);
    }
    if (!hubs.empty()) h.hub_ptr.push_back((int32_t)hubs.size());
    for (size_t i = 0; i + 1 < h.hub_ptr.size(); ++i)
        h.max_hub_len = std::max(h.max_hub_len, h.hub_ptr[i + 1] - h.hub_ptr[i]);
    if ((int64_t)h.max_hub_len > (int64_t)HUB_K * HUB_MAX_CHUNKS)
        return {CS_ENOTSUP, "a hub entry has more contributions than the reduction supports"};
    h.hub_cptr.assign(1, 0);
    h.hub_of_chunk.clear();
    for (size_t i = 0; i + 1 < h.hub_ptr.size(); ++i) {
        const int32_t m = h.hub_ptr[i + 1] - h.hub_ptr[i];
        const int32_t nc = (m + HUB_K - 1) / HUB_K;
        for (int32_t j = 0; j < nc; ++j) h.hub_of_chunk.push_back((int32_t)i);
        h.hub_cptr.push_back(h.hub_cptr.back() + nc);
    }

    // fixed stores: voltage-source stamps, then every entry without a writer
    h.fixA_idx.clear(); h.fixA_val.clear(); h.fixB_idx.clear(); h.fixB_val.clear();
    for (int32_t j = 0; j < h.n_vsrc; ++j) {
        const int32_t br = n_node_rows + j;
        for (int e = 0; e < 2; ++e) {
            int32_t nd = h.vsrc[2 * (size_t)j + e];
            if (nd == 0) continue;
            const double sgn = e == 0 ? 1.0 : -1.0;
            for (int32_t s : {slot_of(nd - 1, br), slot_of(br, nd - 1)}) {
                if (wrote_A[(size_t)s] == -2) continue;
                h.fixA_idx.push_back(s);
                h.fixA_val.push_back(sgn);
                wrote_A[(size_t)s] = -2;
            }
        }
        h.fixB_idx.push_back(br);
        h.fixB_val.push_back(h.vsrc_volts[(size_t)j]);
        wrote_b[(size_t)br] = -2;
    }
    // linear part of the series resistors: +g on the two diagonals, -g between the
    // nodes, summed per entry in resistor order from zero.  It is added once after the
    // device contributions: as the fixed store (0 + part) of an entry no device
    // writes, else by the linear-add pass that follows every schedule.
    std::vector<double> lin;
    std::vector<uint8_t> lin_on;
    if (n_res) {
        lin.assign((size_t)h.nnz, 0.0);
        lin_on.assign((size_t)h.nnz, 0);
        for (size_t j = 0; j < n_res; ++j) {
            const int32_t nd[2] = {h.res[2 * j], h.res[2 * j + 1]};
            for (int r = 0; r < 2; ++r)
                for (int c = 0; c < 2; ++c) {
                    if (nd[r] == 0 || nd[c] == 0) continue;
                    const int32_t s = slot_of(nd[r] - 1, nd[c] - 1);
                    lin[(size_t)s] = lin[(size_t)s] + (r == c ? h.res_g[j] : -h.res_g[j]);
                    lin_on[(size_t)s] = 1;
                }
        }
    }
    h.linA_idx.clear(); h.linA_val.clear();
    for (int64_t s = 0; s < h.nnz; ++s) {
        const bool on = n_res && lin_on[(size_t)s];
        if (wrote_A[(size_t)s] == -1) {
            h.fixA_idx.push_back((int32_t)s);
            h.fixA_val.push_back(on ? 0.0 + lin[(size_t)s] : 0.0);
        } else if (on) {
            h.linA_idx.push_back((int32_t)s);
            h.linA_val.push_back(lin[(size_t)s]);
        }
    }
    for (int64_t r = 0; r < n_rows; ++r)
        if (wrote_b[(size_t)r] == -1) { h.fixB_idx.push_back((int32_t)r); h.fixB_val.push_back(0.0); }
    h.mapped = true;
    return {CS_OK, ""};
}

DevCard derive_card(const cs_model_card &c) {
    // CODATA 2018 / SI exact constants
    const double EPS0 = 8.8541878128e-12, QE = 1.602176634e-19, KB_Q = 8.617333262e-5;
    DevCard d;
    std::memset(&d, 0, sizeof(d));
    d.VT = KB_Q * c.tnom;
    const double EPSOX = 3.9 * EPS0;
    const double EPSSI = 11.7 * EPS0;
    d.COXE = EPSOX / c.toxe;
    const double XDEP0 = std::sqrt(((2.0 * EPSSI) * c.phis) / (QE * c.ndep));
    d.LT = std::sqrt(((EPSSI * c.toxe) * XDEP0) / EPSOX);
    const double CDEP0 = EPSSI / XDEP0;
    const double KS = std::sqrt((2.0 * c.phis) / ((QE * EPSSI) * c.ndep));
    d.LA = 2.0 * std::sqrt(c.xj * XDEP0);
    d.SQPHIS = std::sqrt(c.phis);
    d.VBM = 0.95 * c.phis;
    d.NCDEP = (c.nfactor * (CDEP0 * d.SQPHIS)) / d.COXE;
    d.INV_TOXE = 1.0 / c.toxe;
    d.COXE_KS = d.COXE * KS;
    d.TWO_VT = 2.0 * d.VT;
    d.FOUR_DELTA = 4.0 * c.delta;
    d.FOUR_DELTA1_VBM = (4.0 * c.delta1) * d.VBM;
    d.VBI_M_PHIS = c.vbi - c.phis;
    d.K3_TOXE_PHIS = (c.k3 * c.toxe) * c.phis;
    d.TWO_WINT = 2.0 * c.wint;
    d.TWO_LINT = 2.0 * c.lint;
    d.TWO_VSAT = 2.0 * c.vsat;
    d.phis = c.phis; d.k1 = c.k1; d.k2 = c.k2; d.eta0 = c.eta0; d.nfactor = c.nfactor;
    d.cdsc = c.cdsc; d.voff = c.voff; d.u0 = c.u0; d.ua = c.ua; d.ub = c.ub; d.uc = c.uc;
    d.toxe = c.toxe; d.delta = c.delta; d.delta1 = c.delta1; d.dvt0 = c.dvt0; d.dvt1 = c.dvt1;
    d.dsub = c.dsub; d.w0 = c.w0; d.lambda_l = c.lambda_l; d.a0 = c.a0; d.cgdo = c.cgdo;
    // junctions: constants in the operation order of the junction equations
    d.jmod = c.jmod != 0.0 ? 1.0 : 0.0;
    d.js = c.js; d.cj = c.cj; d.pb = c.pb; d.hdif = c.hdif; d.vjmax = c.vjmax;
    d.NJ_VT = c.nj * d.VT;
    d.FCPB = c.fc * c.pb;
    d.FCPB2 = d.FCPB * d.FCPB;
    d.TWO_PB = 2.0 * c.pb;
    d.QUARTER_PB = 0.25 / c.pb;
    const double s1 = std::sqrt(1.0 - c.fc);
    d.JF1 = (2.0 * c.pb) * (1.0 - s1);
    d.JF2 = (1.0 - c.fc) * s1;
    d.JF3 = 1.0 - 1.5 * c.fc;
    return d;
}

}  // namespace cs
