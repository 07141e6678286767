// Region schedule, host planner.
//
// The colour order of the paper's schedule (Methodology: colours processed in
// sequence, a colour's devices in parallel) fixes, for every matrix entry and RHS
// row, the order in which its writers accumulate: the writer of the smallest colour
// stores, the others add in ascending colour.  The region schedule keeps exactly
// that per-entry order but runs it at workgroup scope:
//   * devices are cut, in ascending device index, into regions of at most one
//     workgroup (a circuit that fits one region is never split);
//   * an entry whose writers all lie in one region and are at most LDS_WRITERS_MAX
//     (one or two) is accumulated in that workgroup's LDS by LDS atomic adds, all
//     writers at once (two values added to the -0.0 start give the same bits in
//     either order); the plan also gives each device a phase, two writers of an
//     entry in distinct phases: an order in which plain loads and stores would do,
//     which the host replay of the plan follows;
//   * an entry whose writers all lie in one region and are more is a lane fold: one
//     lane folds the writers' merged values, read from LDS in colour order, and
//     stores the result (no phase per writer); so are single-writer entries of a
//     region whose LDS slots would not fit the workgroup's LDS (one lane stores the
//     writer's value);
//   * an entry written from several regions has its contributions staged, in colour
//     order, in a global array; the last of its regions to finish (a counter) folds
//     them left and stores the result, or, for entries with more than ITEM_LANE_MAX
//     contributions, a follow-up kernel folds them (one wave per entry);
//   * hub entries keep their fixed-shape sum: contributions staged in ascending
//     device index, each aligned chunk of HUB_K summed by the pairwise tree by the
//     last region touching it, the chunk sums by the same tree.
// The result is bitwise the colour-order accumulation.
#include <algorithm>
#include <numeric>

#include "internal.hpp"

namespace cs {

namespace {

int distinct_k(const std::vector<int32_t> &term, size_t n, size_t p) {
    int32_t u[4];
    int k = 0;
    for (int t = 0; t < 4; ++t) {
        const int32_t nd = term[(size_t)t * n + p];
        if (nd == 0) continue;
        bool seen = false;
        for (int j = 0; j < k; ++j) seen = seen || u[j] == nd;
        if (!seen) u[k++] = nd;
    }
    return k;
}

inline int lanes_needed(int nN, int nP) { return nN + nP; }

}  // namespace

Err build_regions(const RegionSource &s, int32_t cap, RegionPlan &R) {
    const size_t n = (size_t)s.n;
    const int64_t nnz = s.nnz, nkeys = s.nnz + s.n_rows;
    if (cap < 64 || cap % 64 != 0) return {CS_EINVAL, "region capacity must be a multiple of 64"};
    R = RegionPlan{};
    R.cap = cap;

    std::vector<int32_t> pos_of(n);
    for (size_t p = 0; p < n; ++p) pos_of[(size_t)s.perm[p]] = (int32_t)p;
    std::vector<int8_t> kk(n);
    for (size_t p = 0; p < n; ++p) {
        kk[p] = (int8_t)distinct_k(s.term, n, p);
        R.max_nc = std::max<int32_t>(R.max_nc, kk[p] * kk[p] + kk[p]);
    }

    // 1. regions over ascending (global) device index
    std::vector<int32_t> region_of(n, 0);
    {
        std::vector<int64_t> gptr = s.group_ptr;
        if (gptr.empty()) gptr = {0, (int64_t)n};
        int32_t r = -1;
        int nN = 0, nP = 0;
        for (size_t gi = 0; gi + 1 < gptr.size(); ++gi) {
            const int64_t g0 = gptr[gi], g1 = gptr[gi + 1];
            int gN = 0, gP = 0;
            for (int64_t g = g0; g < g1; ++g) (s.pol[(size_t)pos_of[(size_t)g]] > 0 ? gN : gP)++;
            // a circuit that fits one region is not split: open a fresh one for it
            if (g1 > g0 && r >= 0 && lanes_needed(gN, gP) <= cap && lanes_needed(nN + gN, nP + gP) > cap) {
                ++r;
                nN = nP = 0;
            }
            for (int64_t g = g0; g < g1; ++g) {
                const bool isN = s.pol[(size_t)pos_of[(size_t)g]] > 0;
                if (r < 0 || lanes_needed(nN + (isN ? 1 : 0), nP + (isN ? 0 : 1)) > cap) {
                    ++r;
                    nN = nP = 0;
                }
                region_of[(size_t)g] = r;
                (isN ? nN : nP)++;
            }
        }
        R.n_regions = r + 1;
        // wave quantisation: regions are dispatched round-robin over the compute
        // units, so when the last round of full regions reaches only a few of them
        // (the chain: 782 regions of 256 on 256 units, 14 units with a fourth), those
        // units' late waves finish last; cutting that round into one-wave regions
        // spreads the same waves over up to four times as many units
        R.cus = s.cus;
        const int32_t tail = s.cus > 0 ? R.n_regions % s.cus : 0;
        if (s.group_ptr.size() <= 2 && cap > 64 && R.n_regions > s.cus && tail > 0 && 4 * tail <= s.cus) {
            const int32_t first = R.n_regions - tail;
            int32_t rr = first - 1;
            int used = 64;
            for (size_t g = 0; g < n; ++g) {
                if (region_of[g] < first) continue;
                if (used == 64) {
                    ++rr;
                    used = 0;
                }
                region_of[g] = rr;
                ++used;
            }
            R.n_regions = rr + 1;
        }
    }

    // 2. writers of every non-hub target (A slot, or nnz + b row), sorted by colour
    std::vector<int64_t> kptr((size_t)nkeys + 1, 0);
    auto target_of = [&](size_t p, int j, uint32_t c) -> int64_t {
        const int k = kk[p];
        const int64_t idx = (int64_t)(c & 0x3FFFFFFFu);
        return j < k * k ? idx : nnz + idx;
    };
    for (size_t p = 0; p < n; ++p) {
        const int k = kk[p];
        for (int j = 0; j < k * k + k; ++j) {
            const uint32_t c = (uint32_t)s.code[(size_t)j * n + p];
            if ((c >> 30) == TAG_HUB) continue;
            kptr[(size_t)target_of(p, j, c) + 1]++;
        }
    }
    for (int64_t t = 0; t < nkeys; ++t) kptr[(size_t)t + 1] += kptr[(size_t)t];
    std::vector<int64_t> wr((size_t)kptr[(size_t)nkeys]);
    {
        std::vector<int64_t> fill(kptr.begin(), kptr.end() - 1);
        for (size_t p = 0; p < n; ++p) {
            const int k = kk[p];
            for (int j = 0; j < k * k + k; ++j) {
                const uint32_t c = (uint32_t)s.code[(size_t)j * n + p];
                if ((c >> 30) == TAG_HUB) continue;
                wr[(size_t)fill[(size_t)target_of(p, j, c)]++] = ((int64_t)p << 5) | j;
            }
        }
    }
    for (int64_t t = 0; t < nkeys; ++t) {
        std::sort(wr.begin() + kptr[(size_t)t], wr.begin() + kptr[(size_t)t + 1],
                  [&](int64_t a, int64_t b) { return s.colour[(size_t)(a >> 5)] < s.colour[(size_t)(b >> 5)]; });
    }

    // new codes, indexed like s.code (colour-major positions)
    std::vector<int32_t> code(s.code.size(), 0);
    std::vector<std::vector<int64_t>> interior((size_t)R.n_regions);
    std::vector<std::vector<int32_t>> rit((size_t)R.n_regions);
    std::vector<uint8_t> is_interior((size_t)nkeys, 0);
    std::vector<std::vector<int64_t>> lfold((size_t)R.n_regions);
    int64_t cursor = s.stage_base;
    std::vector<int32_t> regs;
    // per staged slot of a shared entry (from stage_base on): target, first writer or
    // not, and the writer's position; hub slots below stage_base
    std::vector<int32_t> slot_tgt((size_t)s.stage_base, -1), slot_pos((size_t)s.stage_base, -1);
    std::vector<uint8_t> slot_first((size_t)s.stage_base, SLOT_HUB);
    for (int64_t t = 0; t < nkeys; ++t) {
        const int64_t b0 = kptr[(size_t)t], b1 = kptr[(size_t)t + 1];
        if (b0 == b1) continue;
        regs.clear();
        for (int64_t w = b0; w < b1; ++w) regs.push_back(region_of[(size_t)s.perm[(size_t)(wr[(size_t)w] >> 5)]]);
        std::sort(regs.begin(), regs.end());
        regs.erase(std::unique(regs.begin(), regs.end()), regs.end());
        if (regs.size() == 1 && b1 - b0 <= LDS_WRITERS_MAX) {
            interior[(size_t)regs[0]].push_back(t);
            is_interior[(size_t)t] = 1;
            continue;
        }
        if (regs.size() == 1) {
            // lane fold: the writers keep their merged values in LDS (code tag 3)
            lfold[(size_t)regs[0]].push_back(t);
            for (int64_t w = b0; w < b1; ++w)
                code[(size_t)(wr[(size_t)w] & 31) * n + (size_t)(wr[(size_t)w] >> 5)] = (int32_t)(3u << 30);
            continue;
        }
        if (cursor + (b1 - b0) >= INDEX_LIMIT) return {CS_ENOTSUP, "too many staged contributions"};
        const int32_t it = (int32_t)(R.item.size() / 4);
        const uint32_t tgt = t < nnz ? (uint32_t)t : ((uint32_t)(t - nnz) | (ITEM_B << 30));
        // large shared entries are folded by the follow-up kernel (regions = 0, no
        // arrival counting); the last arriving region would otherwise fold many
        const bool deferred = b1 - b0 > ITEM_LANE_MAX;
        R.item.insert(R.item.end(), {(int32_t)cursor, (int32_t)(b1 - b0), (int32_t)tgt,
                                     deferred ? 0 : (int32_t)regs.size()});
        if (deferred) R.deferred.push_back(it);
        else
            for (int32_t g : regs) rit[(size_t)g].push_back(it);
        for (int64_t w = b0; w < b1; ++w) {
            const size_t p = (size_t)(wr[(size_t)w] >> 5);
            const int j = (int)(wr[(size_t)w] & 31);
            code[(size_t)j * n + p] = (int32_t)((TAG_STAGE << 30) | (uint32_t)(cursor + (w - b0)));
            slot_tgt.push_back((int32_t)tgt);
            slot_first.push_back(deferred ? SLOT_DEFER : w == b0 ? SLOT_STORE : SLOT_ADD);
            slot_pos.push_back((int32_t)p);
        }
        cursor += b1 - b0;
    }
    R.stage_size = cursor;

    // 3. hub contributions, in the region schedule's parts: chunks of RHUB_K (aligned
    // blocks of the pairwise tree, so each is a subtree).  A part whose contributions
    // all come from one region is a candidate for that region's LDS (step 4b); a part
    // spanning regions keeps its staging indices and is an item, summed by the last of
    // its regions.
    std::vector<std::vector<int32_t>> lchunk((size_t)R.n_regions);          // local parts
    std::vector<std::vector<int32_t>> cand((size_t)R.n_regions);            // candidates
    std::vector<std::vector<std::pair<int32_t, int64_t>>> csrc;   // per part: (staging index, p << 5 | j)
    // one part as an item over its staged contributions
    auto stage_part = [&](size_t q) {
        const auto &v = csrc[q];
        const int32_t h = R.hub_of_chunk[q];
        const int32_t beg = s.hub_ptr[(size_t)h] + (int32_t)(q - (size_t)R.hub_cptr[(size_t)h]) * RHUB_K;
        std::vector<int32_t> rg;
        for (const auto &e : v) {
            code[(size_t)(e.second & 31) * n + (size_t)(e.second >> 5)] = (int32_t)((TAG_STAGE << 30) | (uint32_t)e.first);
            rg.push_back(region_of[(size_t)s.perm[(size_t)(e.second >> 5)]]);
        }
        std::sort(rg.begin(), rg.end());
        rg.erase(std::unique(rg.begin(), rg.end()), rg.end());
        const int32_t it = (int32_t)(R.item.size() / 4);
        R.item.insert(R.item.end(), {beg, (int32_t)v.size(), (int32_t)((ITEM_HUB << 30) | (uint32_t)q), (int32_t)rg.size()});
        for (int32_t g : rg) rit[(size_t)g].push_back(it);
    };
    {
        const int32_t nh = s.hub_ptr.empty() ? 0 : (int32_t)s.hub_ptr.size() - 1;
        R.hub_cptr.assign(1, 0);
        R.hub_of_chunk.clear();
        for (int32_t h = 0; h < nh; ++h) {
            const int32_t m = s.hub_ptr[(size_t)h + 1] - s.hub_ptr[(size_t)h];
            const int32_t nc = (m + RHUB_K - 1) / RHUB_K;
            if (nc > HUB_MAX_PARTS) return {CS_ENOTSUP, "a hub entry has more contributions than the reduction supports"};
            for (int32_t j = 0; j < nc; ++j) R.hub_of_chunk.push_back(h);
            R.hub_cptr.push_back(R.hub_cptr.back() + nc);
        }
        const size_t nparts = R.hub_of_chunk.size();
        csrc.resize(nparts);
        std::vector<int32_t> owner(nparts, -1);   // region of the part's contributions, -2 several
        for (size_t p = 0; p < n; ++p) {
            const int k = kk[p];
            for (int j = 0; j < k * k + k; ++j) {
                const uint32_t c = (uint32_t)s.code[(size_t)j * n + p];
                if ((c >> 30) != TAG_HUB) continue;
                const int32_t si = (int32_t)(c & 0x3FFFFFFFu);
                const size_t h = (size_t)(std::upper_bound(s.hub_ptr.begin(), s.hub_ptr.end(), si) - s.hub_ptr.begin()) - 1;
                const int32_t q = R.hub_cptr[h] + (si - s.hub_ptr[h]) / RHUB_K;
                const int32_t g = region_of[(size_t)s.perm[p]];
                owner[(size_t)q] = owner[(size_t)q] == -1 || owner[(size_t)q] == g ? g : -2;
                csrc[(size_t)q].emplace_back(si, ((int64_t)p << 5) | j);
            }
        }
        for (size_t q = 0; q < nparts; ++q) {
            auto &v = csrc[q];
            std::sort(v.begin(), v.end());
            const int32_t h = R.hub_of_chunk[q];
            const int32_t beg = s.hub_ptr[(size_t)h] + (int32_t)(q - (size_t)R.hub_cptr[(size_t)h]) * RHUB_K;
            const int32_t cnt = std::min<int32_t>(RHUB_K, s.hub_ptr[(size_t)h + 1] - beg);
            if ((int32_t)v.size() != cnt) return {CS_EINVAL, "hub contributions do not fill their staging range"};
            if (owner[q] >= 0) {
                // candidate: code decided in step 4b (tag 3 meanwhile: no LDS slot)
                for (const auto &e : v) code[(size_t)(e.second & 31) * n + (size_t)(e.second >> 5)] = (int32_t)(3u << 30);
                cand[(size_t)owner[q]].push_back((int32_t)q);
                continue;
            }
            stage_part(q);
        }
    }

    // 3b. LDS budget: a region whose owned entries would not fit the workgroup's LDS
    // next to the merged-value rows hands single-writer entries to lane folds
    {
        const int64_t rows = (int64_t)R.max_nc * cap;
        const int64_t budget = REGION_LDS_LIMIT / 8 - rows - 2;
        for (int32_t g = 0; g < R.n_regions; ++g) {
            auto &v = interior[(size_t)g];
            int64_t excess = (int64_t)v.size() - budget;
            if (excess <= 0) continue;
            std::vector<int64_t> keep;
            for (int64_t t : v) {
                const int64_t w0 = kptr[(size_t)t];
                if (excess > 0 && kptr[(size_t)t + 1] - w0 == 1) {
                    lfold[(size_t)g].push_back(t);
                    is_interior[(size_t)t] = 0;
                    code[(size_t)(wr[(size_t)w0] & 31) * n + (size_t)(wr[(size_t)w0] >> 5)] = (int32_t)(3u << 30);
                    --excess;
                } else {
                    keep.push_back(t);
                }
            }
            v.swap(keep);
        }
    }

    // 4. LDS slots of the interior entries (sorted by target) and their codes
    std::vector<int32_t> lds_of((size_t)nkeys, -1);
    std::vector<int32_t> int_ptr((size_t)R.n_regions + 1, 0);
    for (int32_t g = 0; g < R.n_regions; ++g) {
        auto &v = interior[(size_t)g];
        std::sort(v.begin(), v.end());
        for (size_t i = 0; i < v.size(); ++i) {
            lds_of[(size_t)v[i]] = (int32_t)i;
            R.int_target.push_back(v[i] < nnz ? (int32_t)v[i] : (int32_t)((uint32_t)(v[i] - nnz) | (ITEM_B << 30)));
        }
        int_ptr[(size_t)g + 1] = (int32_t)R.int_target.size();
        R.max_lds = std::max<int32_t>(R.max_lds, (int32_t)v.size());
        std::vector<int64_t>().swap(v);
    }
    for (int64_t t = 0; t < nkeys; ++t) {
        if (!is_interior[(size_t)t]) continue;
        for (int64_t w = kptr[(size_t)t]; w < kptr[(size_t)t + 1]; ++w) {
            const size_t p = (size_t)(wr[(size_t)w] >> 5);
            const int j = (int)(wr[(size_t)w] & 31);
            const uint32_t tag = w == kptr[(size_t)t] ? TAG_LDS_STORE : TAG_LDS_ADD;
            code[(size_t)j * n + p] = (int32_t)((tag << 30) | (uint32_t)lds_of[(size_t)t]);
        }
    }

    // 4b. local hub parts: RHUB_K LDS slots each after the region's owned entries (the
    // unused ones stay at their -0.0 start), one writer per slot (plain store, in the
    // writer's phase), when they fit the workgroup's LDS next to the merged-value rows;
    // otherwise the region's candidates are staged items of that region alone
    {
        const int64_t budget = REGION_LDS_LIMIT / 8 - (int64_t)R.max_nc * cap - 2;
        for (int32_t g = 0; g < R.n_regions; ++g) {
            auto &cv = cand[(size_t)g];
            if (cv.empty()) continue;
            const int64_t base = int_ptr[(size_t)g + 1] - int_ptr[(size_t)g];
            if (base + (int64_t)RHUB_K * (int64_t)cv.size() > budget) {
                for (int32_t q : cv) stage_part((size_t)q);
                continue;
            }
            for (size_t k = 0; k < cv.size(); ++k) {
                const int32_t q = cv[k];
                const int32_t h = R.hub_of_chunk[(size_t)q];
                const int32_t start = s.hub_ptr[(size_t)h] + (q - R.hub_cptr[(size_t)h]) * RHUB_K;
                for (const auto &e : csrc[(size_t)q]) {
                    const uint32_t slot = (uint32_t)(base + (int64_t)RHUB_K * (int64_t)k + (e.first - start));
                    code[(size_t)(e.second & 31) * n + (size_t)(e.second >> 5)] = (int32_t)((TAG_LDS_STORE << 30) | slot);
                }
                lchunk[(size_t)g].push_back(q);
            }
            R.max_lds = std::max<int32_t>(R.max_lds, (int32_t)(base + (int64_t)RHUB_K * (int64_t)cv.size()));
        }
    }

    // 5. levels: devices of a region in colour order; a device comes one level after
    // the previous writer of each of its interior entries with three or more
    // writers, and at another level than the other writer of each two-writer entry
    // (two contributions added to the -0.0 start give the same bits in either order)
    std::vector<int32_t> level(n, 0), nphase((size_t)R.n_regions, 0);
    {
        std::vector<int32_t> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
            const int32_t ra = region_of[(size_t)s.perm[(size_t)a]], rb = region_of[(size_t)s.perm[(size_t)b]];
            return ra != rb ? ra < rb : s.colour[(size_t)a] < s.colour[(size_t)b];
        });
        std::vector<int32_t> last((size_t)nkeys, -1);
        std::vector<int32_t> avoid;
        for (int32_t p : order) {
            const int k = kk[(size_t)p];
            int32_t lv = 0;
            avoid.clear();
            for (int j = 0; j < k * k + k; ++j) {
                const uint32_t c = (uint32_t)s.code[(size_t)j * n + (size_t)p];
                if ((c >> 30) == TAG_HUB) continue;
                const int64_t t = target_of((size_t)p, j, c);
                if (!is_interior[(size_t)t]) continue;
                if (kptr[(size_t)t + 1] - kptr[(size_t)t] == 2) {
                    if (last[(size_t)t] >= 0) avoid.push_back(last[(size_t)t]);
                } else {
                    lv = std::max(lv, last[(size_t)t] + 1);
                }
            }
            std::sort(avoid.begin(), avoid.end());
            for (int32_t a : avoid)
                if (a == lv) ++lv;
            for (int j = 0; j < k * k + k; ++j) {
                const uint32_t c = (uint32_t)s.code[(size_t)j * n + (size_t)p];
                if ((c >> 30) == TAG_HUB) continue;
                const int64_t t = target_of((size_t)p, j, c);
                if (is_interior[(size_t)t]) last[(size_t)t] = lv;
            }
            level[(size_t)p] = lv;
            const int32_t g = region_of[(size_t)s.perm[(size_t)p]];
            nphase[(size_t)g] = std::max(nphase[(size_t)g], lv + 1);
        }
    }

    // 5b. global levels of the shared entries (grid-barrier schedule): a device's level
    // is one more than the largest level of the previous writer (in colour order) of
    // any of its shared entries; devices visited in colour order
    std::vector<int32_t> glevel(n, 0);
    R.max_glevel = 0;
    {
        std::vector<int32_t> order(n);
        std::iota(order.begin(), order.end(), 0);
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return s.colour[(size_t)a] < s.colour[(size_t)b]; });
        bool any = false;
        for (int32_t p : order) {
            const int k = kk[(size_t)p];
            int32_t lv = 0;
            bool shared = false;
            for (int j = 0; j < k * k + k; ++j) {
                const uint32_t c = (uint32_t)code[(size_t)j * n + (size_t)p];
                if ((c >> 30) != TAG_STAGE) continue;
                const int64_t sl = (int64_t)(c & 0x3FFFFFFFu);
                if (sl < s.stage_base || slot_first[(size_t)sl] == SLOT_DEFER) continue;
                shared = true;
                if (slot_first[(size_t)sl] == SLOT_ADD) lv = std::max(lv, glevel[(size_t)slot_pos[(size_t)sl - 1]] + 1);
            }
            glevel[(size_t)p] = lv;
            if (shared) {
                any = true;
                R.max_glevel = std::max(R.max_glevel, lv + 1);
            }
        }
        (void)any;
        // beyond 16-bit levels the grid-barrier form is unavailable (the workgroup
        // schedule does not use the levels); -1 marks that
        if (R.max_glevel > 65535) {
            R.max_glevel = -1;
            std::fill(glevel.begin(), glevel.end(), 0);
        }
    }
    R.slot_tgt = std::move(slot_tgt);
    R.slot_first = std::move(slot_first);

    // 6. region-major positions: per region its NMOS, then its PMOS, each in phase
    // order (so that a wave's lanes mostly share one phase), then device order
    R.perm.resize(n);
    R.cm_pos.resize(n);
    R.term.assign(4 * n, 0);
    R.pol.assign(n, 0);
    R.phase.assign(n, 0);
    R.glevel.assign(n, 0);
    R.code.assign((size_t)NCODE * n, (int32_t)(3u << 30));
    R.rtab.assign((size_t)R.n_regions * RT_FIELDS, 0);
    {
        std::vector<std::vector<int32_t>> members((size_t)R.n_regions);
        for (size_t g = 0; g < n; ++g) members[(size_t)region_of[g]].push_back((int32_t)g);
        for (auto &mv : members)
            std::stable_sort(mv.begin(), mv.end(), [&](int32_t a, int32_t b) {
                return level[(size_t)pos_of[(size_t)a]] < level[(size_t)pos_of[(size_t)b]];
            });
        size_t q = 0;
        for (int32_t g = 0; g < R.n_regions; ++g) {
            int32_t *rt = &R.rtab[(size_t)g * RT_FIELDS];
            rt[0] = (int32_t)q;
            int nN = 0, nP = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int32_t dv : members[(size_t)g]) {
                    const size_t p = (size_t)pos_of[(size_t)dv];
                    const bool isN = s.pol[p] > 0;
                    if (isN != (pass == 0)) continue;
                    (isN ? nN : nP)++;
                    R.perm[q] = dv;
                    R.cm_pos[q] = (int32_t)p;
                    for (int t = 0; t < 4; ++t) R.term[(size_t)t * n + q] = s.term[(size_t)t * n + p];
                    R.pol[q] = s.pol[p];
                    if (level[p] > 65535) return {CS_ENOTSUP, "too many phases in a region"};
                    R.phase[q] = (uint16_t)level[p];
                    R.glevel[q] = (uint16_t)glevel[p];
                    const int k = kk[p];
                    for (int j = 0; j < k * k + k; ++j) R.code[(size_t)j * n + q] = code[(size_t)j * n + p];
                    ++q;
                }
            }
            rt[1] = nN;
            rt[2] = nP;
            rt[3] = nphase[(size_t)g];
            rt[4] = int_ptr[(size_t)g];
            rt[5] = int_ptr[(size_t)g + 1];
            rt[6] = (int32_t)R.ritems.size();
            auto &li = rit[(size_t)g];
            std::sort(li.begin(), li.end());
            R.ritems.insert(R.ritems.end(), li.begin(), li.end());
            rt[7] = (int32_t)R.ritems.size();
            R.max_phase = std::max(R.max_phase, nphase[(size_t)g]);
        }
        // lane folds: per region its entries in target order, each with its writers'
        // (code row, lane) in colour order
        std::vector<int32_t> new_pos(n);
        for (size_t q2 = 0; q2 < n; ++q2) new_pos[(size_t)R.cm_pos[q2]] = (int32_t)q2;
        for (int32_t g = 0; g < R.n_regions; ++g) {
            int32_t *rt = &R.rtab[(size_t)g * RT_FIELDS];
            rt[8] = (int32_t)(R.fold.size() / 3);
            for (int64_t t : lfold[(size_t)g]) {
                const uint32_t tgt = t < nnz ? (uint32_t)t : ((uint32_t)(t - nnz) | (ITEM_B << 30));
                const int64_t b0 = kptr[(size_t)t], b1 = kptr[(size_t)t + 1];
                if ((int64_t)R.fold_src.size() + (b1 - b0) >= INDEX_LIMIT) return {CS_ENOTSUP, "too many lane-fold sources"};
                R.fold.insert(R.fold.end(), {(int32_t)tgt, (int32_t)R.fold_src.size(), (int32_t)(b1 - b0)});
                for (int64_t w = b0; w < b1; ++w) {
                    const size_t p = (size_t)(wr[(size_t)w] >> 5);
                    const int32_t j = (int32_t)(wr[(size_t)w] & 31);
                    R.fold_src.push_back((j << 16) | (new_pos[p] - rt[0]));
                }
            }
            rt[9] = (int32_t)(R.fold.size() / 3);
            // local hub parts (LDS slots in this order after the owned entries)
            rt[10] = (int32_t)R.hfold.size();
            R.hfold.insert(R.hfold.end(), lchunk[(size_t)g].begin(), lchunk[(size_t)g].end());
            rt[11] = (int32_t)R.hfold.size();
        }
    }
    R.built = true;
    return {CS_OK, ""};
}

}  // namespace cs

namespace cs {

hipError_t upload_regions(const RegionPlan &R, RegionDev &D) {
    hipError_t e;
    if ((e = D.perm.upload(R.perm)) != hipSuccess) return e;
    if ((e = D.cm_pos.upload(R.cm_pos)) != hipSuccess) return e;
    if ((e = D.term.upload(R.term)) != hipSuccess) return e;
    if ((e = D.code.upload(R.code)) != hipSuccess) return e;
    if ((e = D.rtab.upload(R.rtab)) != hipSuccess) return e;
    if ((e = D.int_target.upload(R.int_target)) != hipSuccess) return e;
    if ((e = D.ritems.upload(R.ritems)) != hipSuccess) return e;
    if ((e = D.item.upload(R.item)) != hipSuccess) return e;
    if ((e = D.deferred.upload(R.deferred)) != hipSuccess) return e;
    if ((e = D.pol.upload(R.pol)) != hipSuccess) return e;
    if ((e = D.phase.upload(R.phase)) != hipSuccess) return e;
    if ((e = D.glevel.upload(R.glevel)) != hipSuccess) return e;
    if ((e = D.slot_tgt.upload(R.slot_tgt)) != hipSuccess) return e;
    if ((e = D.slot_first.upload(R.slot_first)) != hipSuccess) return e;
    if ((e = D.fold.upload(R.fold)) != hipSuccess) return e;
    if ((e = D.fold_src.upload(R.fold_src)) != hipSuccess) return e;
    {
        const size_t nf = R.fold.size() / 3;
        std::vector<int32_t> head(FOLD_HEAD * nf, 0);
        for (size_t i = 0; i < nf; ++i) {
            const int32_t s0 = R.fold[3 * i + 1], cnt = R.fold[3 * i + 2];
            for (int k = 0; k < FOLD_HEAD && k < cnt; ++k) head[FOLD_HEAD * i + (size_t)k] = R.fold_src[(size_t)s0 + (size_t)k];
        }
        if ((e = D.fold_head.upload(head)) != hipSuccess) return e;
    }
    {
        // an item's count is at most RHUB_K (a hub part) or ITEM_LANE_MAX (a shared
        // entry), and so is the number of regions contributing to it
        static_assert(RHUB_K < (1 << ITEM_NEED_SHIFT) && ITEM_LANE_MAX < (1 << ITEM_NEED_SHIFT) &&
                          RHUB_K < (1 << (31 - ITEM_NEED_SHIFT)), "count and regions share one word");
        std::vector<int32_t> ih(4 * R.ritems.size());
        for (size_t i = 0; i < R.ritems.size(); ++i) {
            const int32_t *f = R.item.data() + 4 * (size_t)R.ritems[i];
            ih[4 * i] = R.ritems[i];
            ih[4 * i + 1] = f[0];
            ih[4 * i + 2] = f[2];
            ih[4 * i + 3] = f[1] | (f[3] << ITEM_NEED_SHIFT);
        }
        if ((e = D.ritem_head.upload(ih)) != hipSuccess) return e;
    }
    if ((e = D.hub_cptr.upload(R.hub_cptr)) != hipSuccess) return e;
    if ((e = D.hub_of_chunk.upload(R.hub_of_chunk)) != hipSuccess) return e;
    if ((e = D.hfold.upload(R.hfold)) != hipSuccess) return e;
    if ((e = D.hub_part.alloc(R.hub_of_chunk.size())) != hipSuccess) return e;
    if ((e = D.sdp.alloc((size_t)NSD * R.perm.size())) != hipSuccess) return e;
    if ((e = D.stage.alloc((size_t)R.stage_size)) != hipSuccess) return e;
    const size_t n_items = R.item.size() / 4;
    if ((e = D.item_count.alloc(n_items * CNT_STRIDE)) != hipSuccess) return e;
    if (n_items && (e = hipMemset(D.item_count.p, 0, sizeof(uint32_t) * D.item_count.n)) != hipSuccess) return e;
    D.sdp_stale = true;
    D.ready = true;
    return hipSuccess;
}

void region_info(const RegionPlan &R, int32_t *n_regions, int32_t *max_phases, int64_t *n_items,
                 int64_t *n_staged, int64_t *n_interior, int64_t *n_links, int64_t *n_folds,
                 int64_t *n_fold_src) {
    if (n_folds) *n_folds = (int64_t)(R.fold.size() / 3);
    if (n_fold_src) *n_fold_src = (int64_t)R.fold_src.size();
    if (n_regions) *n_regions = R.n_regions;
    if (max_phases) *max_phases = R.max_phase;
    if (n_items) *n_items = (int64_t)(R.item.size() / 4);
    if (n_staged) *n_staged = R.stage_size;
    if (n_interior) *n_interior = (int64_t)R.int_target.size();
    if (n_links) *n_links = (int64_t)R.ritems.size();
}

template <class T>
static void copy_out(const std::vector<T> &v, T *dst) {
    if (dst && !v.empty()) std::copy(v.begin(), v.end(), dst);
}

void region_tables(const RegionPlan &R, int32_t *perm, uint16_t *phase, int32_t *code, int32_t *rtab,
                   int32_t *interior, int32_t *links, int32_t *item, int32_t *fold, int32_t *fold_src) {
    copy_out(R.fold, fold);
    copy_out(R.fold_src, fold_src);
    copy_out(R.perm, perm);
    copy_out(R.phase, phase);
    copy_out(R.code, code);
    copy_out(R.rtab, rtab);
    copy_out(R.int_target, interior);
    copy_out(R.ritems, links);
    copy_out(R.item, item);
}

void region_hub_tables(const RegionPlan &R, int64_t *counts, int32_t *hfold, int32_t *part_ptr) {
    if (counts) {
        counts[0] = (int64_t)R.hfold.size();
        counts[1] = R.hub_cptr.empty() ? 0 : (int64_t)R.hub_cptr.size() - 1;
    }
    copy_out(R.hfold, hfold);
    copy_out(R.hub_cptr, part_ptr);
}

KCirc region_kcirc(const KCirc &base, const RegionPlan &R, const RegionDev &D) {
    KCirc k = base;
    k.n = (int32_t)R.perm.size();
    k.n_colors = 0;
    k.term = D.term.p;
    k.pol = D.pol.p;
    k.par = nullptr;
    k.sdp = D.sdp.p;
    k.code = D.code.p;
    k.acode = nullptr;
    k.perm = D.perm.p;
    k.cptr = nullptr;
    k.stage = D.stage.p;
    // hub parts in the region schedule's chunks
    k.n_hub_chunks = (int32_t)R.hub_of_chunk.size();
    k.hub_cptr = D.hub_cptr.p;
    k.hub_of_chunk = D.hub_of_chunk.p;
    k.hub_part = D.hub_part.p;
    k.hub_count = nullptr;   // the region schedule counts no hub arrivals
    return k;
}

KRegion region_kregion(const RegionPlan &R, const RegionDev &D) {
    KRegion r{};
    r.n_regions = R.n_regions;
    r.rtab = D.rtab.p;
    r.phase = D.phase.p;
    r.int_target = D.int_target.p;
    r.ritems = D.ritems.p;
    r.item = D.item.p;
    r.ritem_head = D.ritem_head.p;
    r.item_count = D.item_count.p;
    r.n_deferred = (int32_t)R.deferred.size();
    r.deferred = D.deferred.p;
    r.max_glevel = R.max_glevel;
    r.glevel = D.glevel.p;
    r.slot_tgt = D.slot_tgt.p;
    r.slot_first = D.slot_first.p;
    r.fold = D.fold.p;
    r.fold_src = D.fold_src.p;
    r.fold_head = D.fold_head.p;
    r.hfold = D.hfold.p;

    r.lds_int = (R.max_lds + 1) & ~1;
    r.nc_max = R.max_nc;
    return r;
}

}  // namespace cs
