// Host part of the sparse solve inside the Newton loop: a fill-reducing order of
// the MNA pattern and one LU factorisation with threshold partial pivoting.  The
// GPU then refactors with the same pivots at every iteration (static pivoting, as
// circuit solvers' refactor loops do), so this runs once per pattern.
//
// Order: first every voltage source as a pair, the column of its driven node
// pivoting on the source's branch row (a single unit entry: the node voltage is
// substituted, without fill) and the branch column on the node's row.  A rail
// ordered last instead would carry, down a chain of amplifying stages, a product
// of their gains into its column of U.  Then nested dissection by level structures
// of what remains: rows of very high degree are taken out and ordered last; each
// connected part of the rest is cut at the middle level of a breadth-first level
// structure rooted at a pseudo-peripheral vertex, the two sides are ordered
// recursively and the separating level follows them.  On the chain-like circuits
// here the separators are single nodes and the fill is small.  The alternative is
// minimum degree on the same graph, which fills far less on irregular netlists but
// can leave long dependency chains; factor_mna factors with both orders and keeps
// the one whose level-scheduled refactorisation it estimates to be faster.
//
// LU: left-looking, one column at a time (Gilbert and Peierls): the sparse
// triangular solve with the columns already factored reaches its nonzero pattern by
// depth-first search, then the pivot is the partner row of a source pair when that
// entry is nonzero, else the column's own row when its magnitude is at least PIV_TOL
// of the largest candidate, else the largest.
#include <algorithm>
#include <cmath>
#include <iterator>
#include <set>
#include <cstdint>
#include <string>
#include <vector>

#include "internal.hpp"

namespace cs {

namespace {

constexpr int32_t ND_LEAF = 64;       // parts this small are ordered as they are
constexpr int32_t ND_DEPTH = 64;      // recursion bound (deeper parts: natural order)
constexpr double PIV_TOL = 1e-3;

struct Graph {
    int32_t n;
    std::vector<int32_t> ptr, adj;   // symmetric adjacency without self loops
};

struct Dissect {
    const Graph &g;
    std::vector<int32_t> part, level, out;
    int32_t tag = 0;
    explicit Dissect(const Graph &gr) : g(gr), part((size_t)gr.n, -1), level((size_t)gr.n, -1) {}

    // Breadth-first levels from root inside the vertices carrying `id`; returns the
    // last vertex reached and fills `comp` with the vertices in visiting order.
    int32_t bfs(int32_t root, int32_t id, std::vector<int32_t> &comp, int32_t &depth) {
        comp.clear();
        comp.push_back(root);
        level[(size_t)root] = 0;
        const int32_t seen = -2 - id;   // marks visited in this sweep
        part[(size_t)root] = seen;
        depth = 0;
        for (size_t h = 0; h < comp.size(); ++h) {
            const int32_t v = comp[h];
            for (int32_t e = g.ptr[(size_t)v]; e < g.ptr[(size_t)v + 1]; ++e) {
                const int32_t u = g.adj[(size_t)e];
                if (part[(size_t)u] != id) continue;
                part[(size_t)u] = seen;
                level[(size_t)u] = level[(size_t)v] + 1;
                depth = std::max(depth, level[(size_t)u]);
                comp.push_back(u);
            }
        }
        for (int32_t v : comp) part[(size_t)v] = id;   // restore membership
        return comp.back();
    }

    void order(std::vector<int32_t> verts, int depth_left) {
        if ((int32_t)verts.size() <= ND_LEAF || depth_left == 0) {
            std::sort(verts.begin(), verts.end());
            out.insert(out.end(), verts.begin(), verts.end());
            return;
        }
        const int32_t id = ++tag;
        for (int32_t v : verts) part[(size_t)v] = id;
        std::vector<int32_t> comp;
        std::vector<std::vector<int32_t>> comps;
        for (int32_t v : verts) {
            if (part[(size_t)v] != id) continue;
            int32_t d = 0;
            bfs(v, id, comp, d);
            for (int32_t u : comp) part[(size_t)u] = -1;   // taken
            comps.push_back(comp);
        }
        for (auto &c : comps) {
            if ((int32_t)c.size() <= ND_LEAF) {
                std::sort(c.begin(), c.end());
                out.insert(out.end(), c.begin(), c.end());
                continue;
            }
            const int32_t cid = ++tag;
            for (int32_t v : c) part[(size_t)v] = cid;
            // pseudo-peripheral root: repeat the sweep from the farthest vertex
            int32_t root = *std::min_element(c.begin(), c.end()), d = 0, prev = -1;
            std::vector<int32_t> lv;
            for (int it = 0; it < 4; ++it) {
                const int32_t far = bfs(root, cid, lv, d);
                if (d <= prev) break;
                prev = d;
                if (it < 3) root = far;
            }
            bfs(root, cid, lv, d);
            for (int32_t v : c) part[(size_t)v] = -1;
            if (d < 2) {   // no useful separator
                std::sort(c.begin(), c.end());
                out.insert(out.end(), c.begin(), c.end());
                continue;
            }
            const int32_t mid = d / 2;
            std::vector<int32_t> lo, hi, sep;
            for (int32_t v : c) {
                const int32_t l = level[(size_t)v];
                (l < mid ? lo : (l > mid ? hi : sep)).push_back(v);
            }
            order(std::move(lo), depth_left - 1);
            order(std::move(hi), depth_left - 1);
            std::sort(sep.begin(), sep.end());
            out.insert(out.end(), sep.begin(), sep.end());
        }
    }
};

}  // namespace

// Minimum degree on the graph of the vertices not skipped: repeatedly eliminate a
// vertex of smallest current degree (ties: smallest index), its neighbours becoming
// a clique (explicit elimination graph).
static std::vector<int32_t> md_order(const Graph &g, const std::vector<uint8_t> &skip) {
    const int32_t n = g.n;
    std::vector<std::vector<int32_t>> adj((size_t)n);
    std::set<std::pair<int32_t, int32_t>> pq;
    for (int32_t v = 0; v < n; ++v) {
        if (skip[(size_t)v]) continue;
        for (int32_t e = g.ptr[(size_t)v]; e < g.ptr[(size_t)v + 1]; ++e) adj[(size_t)v].push_back(g.adj[(size_t)e]);
        std::sort(adj[(size_t)v].begin(), adj[(size_t)v].end());
        pq.insert({(int32_t)adj[(size_t)v].size(), v});
    }
    std::vector<int32_t> out, tmp;
    while (!pq.empty()) {
        const int32_t v = pq.begin()->second;
        pq.erase(pq.begin());
        out.push_back(v);
        const std::vector<int32_t> nb = std::move(adj[(size_t)v]);
        adj[(size_t)v].clear();
        for (int32_t u : nb) {
            auto &au = adj[(size_t)u];
            pq.erase({(int32_t)au.size(), u});
            tmp.clear();
            std::set_union(au.begin(), au.end(), nb.begin(), nb.end(), std::back_inserter(tmp));
            tmp.erase(std::remove_if(tmp.begin(), tmp.end(), [&](int32_t w) { return w == u || w == v; }), tmp.end());
            au.swap(tmp);
            pq.insert({(int32_t)au.size(), u});
        }
    }
    return out;
}

MnaView circuit_view(const HostCircuit &h) {
    MnaView m;
    m.n = h.n_rows;
    m.row_ptr = h.row_ptr.data();
    m.col_idx = h.col_idx.data();
    for (int32_t j = 0; j < h.n_vsrc; ++j) {
        const int32_t a = h.vsrc[2 * (size_t)j], b = h.vsrc[2 * (size_t)j + 1];
        m.src.push_back({a - 1, b - 1, h.n_nodes - 1 + j});   // ground -> -1
    }
    return m;
}

void mna_order(const MnaView &m, std::vector<int32_t> &Q, std::vector<int32_t> &pref, int method) {
    const int32_t n = m.n;
    const int32_t *row_ptr = m.row_ptr, *col_idx = m.col_idx;
    Q.clear();
    pref.assign((size_t)n, -1);
    std::vector<uint8_t> taken((size_t)n, 0);
    for (const auto &sr : m.src) {
        const int32_t br = sr[2];
        int32_t nd = sr[0];
        if (nd < 0 || taken[(size_t)nd]) nd = sr[1];
        if (nd < 0 || taken[(size_t)nd]) continue;
        taken[(size_t)nd] = taken[(size_t)br] = 1;
        Q.push_back(nd);
        Q.push_back(br);
        pref[(size_t)nd] = br;
        pref[(size_t)br] = nd;
    }
    // high degree: more than 32 neighbours and more than 8 times the mean
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i) total += row_ptr[i + 1] - row_ptr[i];
    const double mean = n ? (double)total / n : 0.0;
    std::vector<uint8_t> heavy((size_t)n, 0);
    for (int32_t i = 0; i < n; ++i) {
        const int32_t d = row_ptr[(size_t)i + 1] - row_ptr[(size_t)i];
        heavy[(size_t)i] = taken[(size_t)i] || (d > 32 && d > 8.0 * mean);
    }
    Graph g;
    g.n = n;
    g.ptr.assign((size_t)n + 1, 0);
    for (int32_t i = 0; i < n; ++i) {
        int32_t c = 0;
        if (!heavy[(size_t)i])
            for (int32_t e = row_ptr[(size_t)i]; e < row_ptr[(size_t)i + 1]; ++e) {
                const int32_t j = col_idx[(size_t)e];
                c += j != i && !heavy[(size_t)j];
            }
        g.ptr[(size_t)i + 1] = g.ptr[(size_t)i] + c;
    }
    g.adj.resize((size_t)g.ptr[(size_t)n]);
    for (int32_t i = 0; i < n; ++i) {
        if (heavy[(size_t)i]) continue;
        int32_t w = g.ptr[(size_t)i];
        for (int32_t e = row_ptr[(size_t)i]; e < row_ptr[(size_t)i + 1]; ++e) {
            const int32_t j = col_idx[(size_t)e];
            if (j != i && !heavy[(size_t)j]) g.adj[(size_t)w++] = j;
        }
    }
    std::vector<int32_t> order;
    if (method == 1) {
        order = md_order(g, heavy);
    } else {
        Dissect nd(g);
        std::vector<int32_t> light;
        for (int32_t i = 0; i < n; ++i)
            if (!heavy[(size_t)i]) light.push_back(i);
        nd.order(std::move(light), ND_DEPTH);
        order = std::move(nd.out);
    }
    for (int32_t i = 0; i < n; ++i)
        if (heavy[(size_t)i] && !taken[(size_t)i]) order.push_back(i);
    Q.insert(Q.end(), order.begin(), order.end());
}

// Estimated time of the level-scheduled refactorisation and solves of T (microseconds,
// fitted to measurements on MI355X of the per-level kernels): per lower level 4.7, per
// upper level 6.8, and 0.94 per L entry of the longest row of each lower level.  The
// programmed rows and the runs of narrow levels make long chains of one-row levels
// cheaper than this, so the estimate leans to nested dissection; it only ranks the
// two orders.
double lu_cost_estimate(const HostLU &F, int32_t *n_lower, int32_t *n_upper) {
    const int32_t n = (int32_t)F.Tp.size() - 1;
    std::vector<int32_t> lev((size_t)n, 0), ulev((size_t)n, 0), nlo((size_t)n, 0);
    int32_t nl = 0, nu = 0;
    for (int32_t i = 0; i < n; ++i) {
        int32_t m = 0, c = 0;
        for (int32_t p = F.Tp[(size_t)i]; p < F.Tp[(size_t)i + 1]; ++p) {
            const int32_t j = F.Ti[(size_t)p];
            if (j < i) { m = std::max(m, lev[(size_t)j] + 1); ++c; }
        }
        lev[(size_t)i] = m;
        nlo[(size_t)i] = c;
        nl = std::max(nl, m + 1);
    }
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t m = 0;
        for (int32_t p = F.Tp[(size_t)i]; p < F.Tp[(size_t)i + 1]; ++p) {
            const int32_t j = F.Ti[(size_t)p];
            if (j > i) m = std::max(m, ulev[(size_t)j] + 1);
        }
        ulev[(size_t)i] = m;
        nu = std::max(nu, m + 1);
    }
    std::vector<int32_t> maxl((size_t)std::max(nl, 1), 0);
    for (int32_t i = 0; i < n; ++i) maxl[(size_t)lev[(size_t)i]] = std::max(maxl[(size_t)lev[(size_t)i]], nlo[(size_t)i]);
    double sum = 0.0;
    for (int32_t v : maxl) sum += v;
    if (n_lower) *n_lower = nl;
    if (n_upper) *n_upper = nu;
    return 4.7 * nl + 6.8 * nu + 0.94 * sum;
}

Err factor_mna(const MnaView &h, const double *A, HostLU &F, int *method) {
    HostLU best;
    double best_cost = 0.0;
    int best_m = -1;
    Err last{CS_OK, ""};
    for (int m = 0; m < 2; ++m) {
        std::vector<int32_t> Q, pref;
        mna_order(h, Q, pref, m);
        HostLU f;
        last = host_lu(h.n, h.row_ptr, h.col_idx, A, Q, pref, f);
        if (last.st != CS_OK) continue;
        const double cost = lu_cost_estimate(f, nullptr, nullptr);
        if (best_m < 0 || cost < best_cost) {
            best = std::move(f);
            best_cost = cost;
            best_m = m;
        }
    }
    if (best_m < 0) return last;
    F = std::move(best);
    if (method) *method = best_m;
    return {CS_OK, ""};
}

Err host_lu(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
            const std::vector<int32_t> &Q, const std::vector<int32_t> &pref, HostLU &F) {
    // columns of A (CSC) from its rows
    const int64_t nnz = row_ptr[(size_t)n];
    std::vector<int32_t> cp((size_t)n + 1, 0), ri((size_t)nnz);
    std::vector<double> cx((size_t)nnz);
    for (int64_t e = 0; e < nnz; ++e) cp[(size_t)col_idx[(size_t)e] + 1]++;
    for (int32_t j = 0; j < n; ++j) cp[(size_t)j + 1] += cp[(size_t)j];
    {
        std::vector<int32_t> fill(cp.begin(), cp.end() - 1);
        for (int32_t i = 0; i < n; ++i)
            for (int32_t e = row_ptr[(size_t)i]; e < row_ptr[(size_t)i + 1]; ++e) {
                const int32_t w = fill[(size_t)col_idx[(size_t)e]]++;
                ri[(size_t)w] = i;
                cx[(size_t)w] = val[e];
            }
    }
    std::vector<int32_t> Lp(1, 0), Li, Up(1, 0), Ui;
    std::vector<double> Lx, Ux;
    std::vector<int32_t> pinv((size_t)n, -1), mark((size_t)n, -1), next((size_t)n, 0), stack, topo;
    std::vector<double> x((size_t)n, 0.0);
    F.P.assign((size_t)n, -1);
    for (int32_t k = 0; k < n; ++k) {
        const int32_t j = Q[(size_t)k];
        // reach of A(:, j) through the factored columns, in depth-first postorder
        topo.clear();
        for (int32_t e = cp[(size_t)j]; e < cp[(size_t)j + 1]; ++e) {
            const int32_t s = ri[(size_t)e];
            if (mark[(size_t)s] == k) continue;
            mark[(size_t)s] = k;
            stack.assign(1, s);
            next[(size_t)s] = 0;
            while (!stack.empty()) {
                const int32_t v = stack.back();
                const int32_t p = pinv[(size_t)v];
                bool pushed = false;
                if (p >= 0) {
                    for (int32_t q = Lp[(size_t)p] + next[(size_t)v]; q < Lp[(size_t)p + 1]; ++q) {
                        const int32_t r = Li[(size_t)q];
                        next[(size_t)v] = q - Lp[(size_t)p] + 1;
                        if (mark[(size_t)r] == k) continue;
                        mark[(size_t)r] = k;
                        next[(size_t)r] = 0;
                        stack.push_back(r);
                        pushed = true;
                        break;
                    }
                }
                if (!pushed) {
                    stack.pop_back();
                    topo.push_back(v);
                }
            }
        }
        // x = L \ A(:, j) on the reach, in topological order
        for (int32_t v : topo) x[(size_t)v] = 0.0;
        for (int32_t e = cp[(size_t)j]; e < cp[(size_t)j + 1]; ++e) x[(size_t)ri[(size_t)e]] = cx[(size_t)e];
        for (size_t t = topo.size(); t-- > 0;) {
            const int32_t v = topo[t];
            const int32_t p = pinv[(size_t)v];
            if (p < 0) continue;
            const double xv = x[(size_t)v];
            for (int32_t q = Lp[(size_t)p]; q < Lp[(size_t)p + 1]; ++q)
                x[(size_t)Li[(size_t)q]] -= Lx[(size_t)q] * xv;
        }
        // pivot among the rows not yet pivoted
        int32_t best = -1;
        double bmax = 0.0;
        for (int32_t v : topo)
            if (pinv[(size_t)v] < 0 && std::fabs(x[(size_t)v]) > bmax) {
                bmax = std::fabs(x[(size_t)v]);
                best = v;
            }
        if (best < 0 || !std::isfinite(bmax))
            return {CS_EDOMAIN, "singular matrix in the host LU (column " + std::to_string(j) + " at step " +
                                    std::to_string(k) + ")"};
        // a source pair takes its partner whenever that entry is nonzero (a unit
        // branch entry: exact substitution, no Schur update); other columns their
        // own row above the threshold
        int32_t piv = best;
        const bool pair = pref[(size_t)j] >= 0;
        const int32_t w = pair ? pref[(size_t)j] : j;
        if (mark[(size_t)w] == k && pinv[(size_t)w] < 0 &&
            (pair ? x[(size_t)w] != 0.0 : std::fabs(x[(size_t)w]) >= PIV_TOL * bmax))
            piv = w;
        const double pv = x[(size_t)piv];
        pinv[(size_t)piv] = k;
        F.P[(size_t)k] = piv;
        for (int32_t v : topo) {
            if (pinv[(size_t)v] >= 0) {
                Ui.push_back(v);
                Ux.push_back(x[(size_t)v]);
            } else {
                Li.push_back(v);
                Lx.push_back(x[(size_t)v] / pv);
            }
        }
        Lp.push_back((int32_t)Li.size());
        Up.push_back((int32_t)Ui.size());
        if ((int64_t)Li.size() + (int64_t)Ui.size() >= INDEX_LIMIT) return {CS_ENOTSUP, "LU factors too large"};
    }
    // T = (L - I) + U of P A Q, rows in pivot order, columns ascending
    F.Q = Q;
    std::vector<int32_t> cnt((size_t)n + 1, 0);
    for (int32_t k = 0; k < n; ++k) {
        for (int32_t q = Up[(size_t)k]; q < Up[(size_t)k + 1]; ++q) cnt[(size_t)pinv[(size_t)Ui[(size_t)q]] + 1]++;
        for (int32_t q = Lp[(size_t)k]; q < Lp[(size_t)k + 1]; ++q) cnt[(size_t)pinv[(size_t)Li[(size_t)q]] + 1]++;
    }
    for (int32_t r = 0; r < n; ++r) cnt[(size_t)r + 1] += cnt[(size_t)r];
    F.Tp = cnt;
    F.Ti.assign((size_t)cnt[(size_t)n], 0);
    F.Tx.assign((size_t)cnt[(size_t)n], 0.0);
    for (int32_t k = 0; k < n; ++k) {   // ascending k: each row's columns come out sorted
        for (int32_t q = Up[(size_t)k]; q < Up[(size_t)k + 1]; ++q) {
            const int32_t r = pinv[(size_t)Ui[(size_t)q]];
            F.Ti[(size_t)cnt[(size_t)r]] = k;
            F.Tx[(size_t)cnt[(size_t)r]++] = Ux[(size_t)q];
        }
        for (int32_t q = Lp[(size_t)k]; q < Lp[(size_t)k + 1]; ++q) {
            const int32_t r = pinv[(size_t)Li[(size_t)q]];
            F.Ti[(size_t)cnt[(size_t)r]] = k;
            F.Tx[(size_t)cnt[(size_t)r]++] = Lx[(size_t)q];
        }
    }
    return {CS_OK, ""};
}

}  // namespace cs
