"""CPU checks of the region schedule's host planner.

The library's plan tables (regions, phases, stamp codes, shared-entry items) are
replayed here on the host exactly as the region kernels use them, with every device's
local values taken from the oracle; the replayed matrix entries and RHS rows must
equal the oracle's colour-order replay bit for bit.  Structural checks cover the
region layout (NMOS lanes first, then PMOS lanes, capacity), the code
rows, the item bookkeeping and, for batches, that a circuit fitting one region is
never split.  Hub entries are summed in parts of 32 contributions: a part held by one
region from its parked values, a part spanning regions from its staged
contributions; the replay forms every hub's pairwise tree from those parts and
compares it with the oracle's hub entries too."""
import numpy as np
import pytest

from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

NC, PC = G.default_card(1), G.default_card(-1)
AG0 = 1e12


def merged_values(orc, circ, v):
    """Device v's merged contributions in code order (node pairs row-major, then RHS
    rows), from the oracle's local Y and bl."""
    t4 = [int(n) for n in circ.term[v]]
    V = np.array([0.0 if n == 0 else circ.x[n - 1] for n in t4])
    pol = int(circ.pol[v])
    Y, bl, _, _ = orc.device_eval(NC if pol > 0 else PC, pol, circ.W[v], circ.L[v], circ.VTH0[v], V, AG0)
    u = []
    for n in t4:
        if n != 0 and n not in u:
            u.append(n)
    m = []
    for a in u:
        for b in u:
            acc = None
            for t in range(4):
                for s in range(4):
                    if t4[t] == a and t4[s] == b:
                        acc = Y[t, s] if acc is None else acc + Y[t, s]
            m.append(acc)
    for a in u:
        acc = None
        for t in range(4):
            if t4[t] == a:
                acc = bl[t] if acc is None else acc + bl[t]
        m.append(acc)
    return m


def tree(vals, size):
    """Perfect binary tree sum of vals padded with -0.0 to size (a power of two)."""
    v = [float(x) for x in vals] + [-0.0] * (size - len(vals))
    while len(v) > 1:
        v = [v[2 * i] + v[2 * i + 1] for i in range(len(v) // 2)]
    return v[0]


def replay(plan, vals, pol, block, nnz, n_rows):
    """Host replay of the region kernel: returns {('A'|'b', index): value} for every
    non-hub entry the plan owns or shares, and per hub its sum formed from the plan's
    parts ({hub index: value})."""
    code, rtab, phase, perm = plan["code"], plan["rtab"], plan["phase"], plan["perm"]
    n = len(perm)
    stage = np.full(plan["n_staged"], np.nan)
    out = {}
    parts = {}
    seen = np.zeros(n, bool)
    nxt = 0
    for r in range(plan["n_regions"]):
        p0, nN, nP, nph, ib, ie, jb, je, fb, fe, hb, he = (int(v) for v in rtab[r])
        assert p0 == nxt and nN + nP > 0
        nxt = p0 + nN + nP
        assert nN + nP <= block
        pos = list(range(p0, p0 + nN + nP))
        assert all(pol[perm[p]] > 0 for p in pos[:nN]) and all(pol[perm[p]] < 0 for p in pos[nN:])
        # owned entries, then 32 slots per local hub part
        lds = np.full(ie - ib + 32 * (he - hb), np.nan)
        folded = set()
        for i in range(fb, fe):
            _, sb, cnt = (int(v) for v in plan["fold"][i])
            assert cnt == 1 or cnt > 2
            for src in plan["fold_src"][sb:sb + cnt]:
                j, lane = int(src) >> 16, int(src) & 0xFFFF
                assert lane < nN + nP and (j, lane) not in folded
                folded.add((j, lane))
        for p in pos:
            seen[p] = True
            for j, mv in enumerate(vals[perm[p]]):
                c = int(code[j, p]) & 0xFFFFFFFF
                tag, idx = c >> 30, c & 0x3FFFFFFF
                # tag 3 within a device's codes: read by a lane fold of the region
                assert tag in (0, 1, 2) or (tag == 3 and (j, p - p0) in folded)
                if tag == 2:
                    assert np.isnan(stage[idx])
                    stage[idx] = mv
            for j in range(len(vals[perm[p]]), 20):
                assert (int(code[j, p]) & 0xFFFFFFFF) >> 30 == 3
            assert phase[p] < max(nph, 1)
        # the plan's phases: two writers of one entry never share a phase
        written = [set() for _ in range(len(lds))]
        for p in pos:
            for j, mv in enumerate(vals[perm[p]]):
                c = int(code[j, p]) & 0xFFFFFFFF
                tag, idx = c >> 30, c & 0x3FFFFFFF
                if tag in (0, 1):
                    assert phase[p] not in written[idx], "two writers of an entry in one phase"
                    written[idx].add(int(phase[p]))
        assert all(written[:ie - ib])
        # as the kernel: accumulators start at -0.0 and the writers add in whatever
        # order their LDS atomics land (here a seeded shuffle), exact because an
        # entry has at most two writers: -0.0 + a = a and a + b = b + a
        assert all(len(w) <= 2 for w in written[:ie - ib])
        assert all(len(w) <= 1 for w in written[ie - ib:])   # one writer per hub slot
        lds[:] = -0.0
        adds = [(p, j) for p in pos for j in range(len(vals[perm[p]]))]
        for k in np.random.default_rng(r).permutation(len(adds)):
            p, j = adds[k]
            c = int(code[j, p]) & 0xFFFFFFFF
            tag, idx = c >> 30, c & 0x3FFFFFFF
            if tag in (0, 1):
                lds[idx] = lds[idx] + vals[perm[p]][j]
        # local hub parts: slot r of part k holds contribution r (-0.0 beyond the
        # part's contributions), summed by the 32-leaf tree
        for k in range(he - hb):
            q = int(plan["hfold"][hb + k])
            assert q not in parts
            parts[q] = tree(lds[ie - ib + 32 * k: ie - ib + 32 * (k + 1)], 32)
        # lane folds: the writers' merged values, left to right in colour order
        for i in range(fb, fe):
            tg, sb, cnt = (int(v) for v in plan["fold"][i])
            tg &= 0xFFFFFFFF
            srcs = [int(v) for v in plan["fold_src"][sb:sb + cnt]]
            s = vals[perm[p0 + (srcs[0] & 0xFFFF)]][srcs[0] >> 16]
            for src in srcs[1:]:
                s = s + vals[perm[p0 + (src & 0xFFFF)]][src >> 16]
            key = ("b" if tg >> 30 == 1 else "A", tg & 0x3FFFFFFF)
            assert key not in out
            out[key] = s
        for i in range(ie - ib):
            tg = int(plan["interior"][ib + i]) & 0xFFFFFFFF
            key = ("b" if tg >> 30 == 1 else "A", tg & 0x3FFFFFFF)
            assert key not in out
            out[key] = lds[i]
    assert nxt == n and seen.all()
    # items: linked from exactly the regions that contribute
    links = {}
    for r in range(plan["n_regions"]):
        jb, je = int(rtab[r][6]), int(rtab[r][7])
        for it in plan["links"][jb:je]:
            links.setdefault(int(it), []).append(r)
    for it, (beg, cnt, tgt, need) in enumerate(plan["item"]):
        tgt = int(tgt) & 0xFFFFFFFF
        assert not np.isnan(stage[beg:beg + cnt]).any()
        if tgt >> 30 == 2:
            # a hub part spanning regions: its staged contributions by the tree
            q = tgt & 0x3FFFFFFF
            assert len(links.get(it, [])) == need >= 2
            assert 1 <= cnt <= 32 and q not in parts
            parts[q] = tree(stage[beg:beg + cnt], 32)
            continue
        if need == 0:     # large shared entry: folded by the follow-up kernel
            assert it not in links and cnt > 8
        else:
            assert len(links.get(it, [])) == need >= 2 and cnt <= 8
        s = stage[beg]
        for k in range(1, cnt):
            s = s + stage[beg + k]
        key = ("b" if tgt >> 30 == 1 else "A", tgt & 0x3FFFFFFF)
        assert key not in out
        out[key] = s
    # hub staging slots of local parts are never written; every other slot is
    hubs = {}
    pp = plan["part_ptr"]
    for h in range(len(pp) - 1):
        q0, q1 = int(pp[h]), int(pp[h + 1])
        assert all(q in parts for q in range(q0, q1))
        size = 1
        while size < q1 - q0:
            size *= 2
        hubs[h] = tree([parts[q] for q in range(q0, q1)], size)
    assert len(parts) == (int(pp[-1]) if len(pp) else 0)
    return out, hubs


def check_against_oracle(orc, circ, c, exclude, block):
    col, _, _ = orc.colour(circ, exclude)
    rp, ci = orc.pattern(circ)
    A0, b0 = orc.assemble(circ, rp, ci, NC, PC, AG0, col=col, exclude=exclude)
    plan = c.region_plan(block)
    vals = [merged_values(orc, circ, v) for v in range(circ.n_dev)]
    out, hubs = replay(plan, vals, circ.pol, block, len(ci), circ.n_rows)
    # hub entries in ascending target order (A slots, then b rows), as the library
    # numbers them; each equals the oracle's entry bit for bit
    slot, sflag, brow, bflag = orc.stamp_map(circ, rp, ci, col, exclude)
    targets = sorted({int(s) for s, f in zip(slot.ravel(), sflag.ravel()) if f == 2} |
                     {len(ci) + int(r) for r, f in zip(brow.ravel(), bflag.ravel()) if f == 2})
    assert len(targets) == len(hubs)
    for h, tg in enumerate(targets):
        ref = A0[tg] if tg < len(ci) else b0[tg - len(ci)]
        assert np.float64(hubs[h]).view(np.int64) == np.float64(ref).view(np.int64), ("hub", h, hubs[h], ref)
    # a split netlist's series resistors: their linear part follows the schedule
    Lin, touched = orc.linear_stamp(circ, rp, ci)
    for (kind, idx), v in out.items():
        if kind == "A" and touched[idx]:
            v = v + Lin[idx]
        ref = (A0 if kind == "A" else b0)[idx]
        assert np.float64(v).view(np.int64) == np.float64(ref).view(np.int64), (kind, idx, v, ref)
    return plan, out


CASES = [
    ("chain50", lambda: G.workload(0)),
    ("opamp12", lambda: G.draw_params(G.opamp2(12), np.random.default_rng(2), G.W_OPAMP, G.L_OPAMP)),
    ("sram6x5", lambda: G.sram_case(6, 5, 8)),
    ("ring301", lambda: G.draw_params(G.ring_oscillator(301), np.random.default_rng(4), G.W_CHAIN, G.L_CHAIN)),
    ("pchain7x3", lambda: G.draw_params(G.parallel_chain(7, 3), np.random.default_rng(5), G.W_CHAIN, G.L_CHAIN)),
    ("pchain9x20", lambda: G.draw_params(G.parallel_chain(9, 20), np.random.default_rng(6), G.W_CHAIN, G.L_CHAIN)),
    ("random600x6", lambda: G.draw_params(G.random_netlist(600, 6, 21), np.random.default_rng(8), G.W_CHAIN,
                                          G.L_CHAIN)),
    # every net split: almost only single-writer entries, more than one region's LDS
    # holds at 256 devices (one-source lane folds)
    ("adder8r89", lambda: G.draw_params(G.split_nets(G.ripple_adder28(8), "all")[0], np.random.default_rng(7),
                                        G.W_CHAIN, G.L_CHAIN)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("exclude", [True, False])
@pytest.mark.parametrize("block", [64, 128, 256])
def test_region_replay_equals_colour_replay(orc, name, make, exclude, block):
    circ = make()
    c = CS.prepare(circ, exclude)
    plan, out = check_against_oracle(orc, circ, c, exclude, block)
    # every non-hub written entry is owned by a region or shared
    rp, ci = orc.pattern(circ)
    col, _, _ = orc.colour(circ, exclude)
    slot, sflag, brow, bflag = orc.stamp_map(circ, rp, ci, col, exclude)
    written = {("A", int(s)) for s, f in zip(slot.ravel(), sflag.ravel()) if s >= 0 and f != 2}
    written |= {("b", int(r)) for r, f in zip(brow.ravel(), bflag.ravel()) if r >= 0 and f != 2}
    assert set(out) == written


def test_chain_regions_are_contiguous_and_phases_are_colours(orc):
    circ = G.workload(0)
    c = CS.prepare(circ, True)
    plan = c.region_plan(64)
    # 100 devices in regions of 64 consecutive devices
    assert plan["n_regions"] == 2
    assert plan["max_phases"] <= 4
    for r in range(plan["n_regions"]):
        p0, nN, nP = (int(v) for v in plan["rtab"][r][:3])
        devs = sorted(int(v) for v in plan["perm"][p0:p0 + nN + nP])
        assert devs == list(range(devs[0], devs[0] + len(devs)))


def test_sram_levels_are_far_fewer_than_colours(orc):
    # regions of 128 devices hold parts of one cell row: the wordline and bitlines
    # are shared with other regions, and the cell-internal nodes need few levels
    circ = G.sram_case(32, 32, 8)
    c = CS.prepare(circ, True)
    plan = c.region_plan(128)
    assert c.n_colors == 68
    assert plan["max_phases"] <= 6


def test_batch_plan_keeps_small_circuits_whole_and_replays(orc):
    circs = G.batch_sweep(seed=9, n_opamp=12, n_chain=3, n_ring=2, chain_range=(50, 300),
                          ring_range=(31, 201))
    B = CS.Batch([CS.prepare(cc, True) for cc in circs])
    plan = B.region_plan(128)
    region_of = np.zeros(B.n_dev, np.int64)
    for r in range(plan["n_regions"]):
        p0, nN, nP = (int(v) for v in plan["rtab"][r][:3])
        region_of[plan["perm"][p0:p0 + nN + nP]] = r
    for i, cc in enumerate(circs):
        regs = set(region_of[B.dev_off[i]:B.dev_off[i + 1]].tolist())
        nN, nP = int((cc.pol > 0).sum()), int((cc.pol < 0).sum())
        if nN + nP <= 128:
            assert len(regs) == 1, cc.name
    # replay of the packed plan against each circuit's oracle colour replay
    vals, pol = [], np.concatenate([cc.pol for cc in circs])
    for cc in circs:
        vals += [merged_values(orc, cc, v) for v in range(cc.n_dev)]
    out, _ = replay(plan, vals, pol, 128, B.nnz, B.n_rows)
    for i, cc in enumerate(circs):
        col, _, _ = orc.colour(cc, True)
        rp, ci = orc.pattern(cc)
        A0, b0 = orc.assemble(cc, rp, ci, NC, PC, AG0, col=col, exclude=True)
        for (kind, idx), v in out.items():
            lo, hi = ((B.nnz_off[i], B.nnz_off[i + 1]) if kind == "A" else (B.row_off[i], B.row_off[i + 1]))
            if lo <= idx < hi:
                ref = (A0 if kind == "A" else b0)[idx - lo]
                assert np.float64(v).view(np.int64) == np.float64(ref).view(np.int64)


def test_plan_errors(orc):
    c = CS.prepare(G.workload(0), True)
    with pytest.raises(CS.CsError):
        c.region_plan(100)
    with pytest.raises(CS.CsError):
        c.region_plan(512)


def test_strict_chain_vdd_entries_are_deferred():
    # without the rail exclusion every PMOS of a chain writes the vdd diagonal and
    # the vdd RHS row: 70,000 writers each, in colour order; they become deferred
    # items (folded by the follow-up kernel), so they chain no levels
    circ = G.chain_case(70_000, seed=8)
    c = CS.prepare(circ, False)
    assert c.n_colors == 70_001
    plan = c.region_plan(256)
    assert plan["n_regions"] == (circ.n_dev + 255) // 256
    assert plan["max_phases"] <= 130
    it = plan["item"]
    # the vdd diagonal and the vdd RHS row: one writer per PMOS, folded by the
    # follow-up kernel (need 0)
    big = it[it[:, 1] == 70_000]
    assert len(big) == 2 and (big[:, 3] == 0).all()


def test_lane_folds_take_many_writer_entries(orc):
    # 20 inverters per stage: the output node's diagonal has 80 writers inside one
    # region of 256, folded by one lane instead of 80 phases
    circ = G.draw_params(G.parallel_chain(9, 20), np.random.default_rng(6), G.W_CHAIN, G.L_CHAIN)
    c = CS.prepare(circ, True)
    plan = c.region_plan(256)
    assert plan["n_folds"] > 0 and plan["max_phases"] <= 8
    assert int(plan["fold"][:, 2].max()) == 80


def test_regions_with_more_items_than_threads(orc):
    # a random netlist of 2,000 FETs on 800 nodes: few writers per entry, spread over
    # many regions, so a region contributes to more shared entries than it has
    # threads and the region kernel counts its arrivals in several rounds (the GPU
    # parity cases include this netlist at blocks 64, 192 and 256)
    circ = G.draw_params(G.random_netlist(2000, 800, 31), np.random.default_rng(78), G.W_CHAIN, G.L_CHAIN)
    c = CS.prepare(circ, True)
    for block in (64, 192, 256):
        rt = c.region_plan(block)["rtab"]
        assert ((rt[:, 7] - rt[:, 6]) > block).sum() >= rt.shape[0] // 2, block
    check_against_oracle(orc, circ, c, True, 64)


def test_last_round_cut_into_one_wave_regions(orc):
    # 5,000 stages at 256 devices per region: 40 regions; planned for 32 compute
    # units the last round (8 regions, 1,808 devices) becomes 29 regions of at most
    # 64 devices, and the replay still equals the colour replay
    circ = G.chain_case(5000, seed=12)
    c = CS.prepare(circ, True)
    c.set_plan_units(0)
    assert c.region_plan(256)["n_regions"] == 40
    c.set_plan_units(32)
    plan, _ = check_against_oracle(orc, circ, c, True, 256)
    assert plan["n_regions"] == 32 + 29
    sizes = plan["rtab"][:, 1] + plan["rtab"][:, 2]
    assert (sizes[:32] == 256).all() and (sizes[32:] <= 64).all() and sizes.sum() == circ.n_dev
    # fewer regions than units: nothing to cut
    c.set_plan_units(48)
    assert c.region_plan(256)["n_regions"] == 40


def test_lds_budget_moves_single_writer_entries_to_lane_folds(orc):
    circ = G.draw_params(G.split_nets(G.ripple_adder28(8), "all")[0], np.random.default_rng(7),
                         G.W_CHAIN, G.L_CHAIN)
    c = CS.prepare(circ, True)
    small = c.region_plan(128)
    assert small["n_folds"] == 0
    plan = c.region_plan(256)
    assert plan["n_regions"] == 1 and plan["n_folds"] > 0 and (plan["fold"][:, 2] == 1).all()
    # slots left in LDS: at most 64 KiB - 1 KiB with the 20 x 256 merged-value rows
    assert plan["n_interior"] + 20 * 256 + 2 <= (65536 - 1024) // 8


def test_chain_hub_parts_are_summed_inside_regions(orc):
    # regions of 256 devices hold 128 PMOS, i.e. four whole parts of 32 contributions
    # of each rail hub (the vdd diagonal and the vdd RHS row): no hub part is staged
    circ = G.chain_case(5000, seed=12)
    c = CS.prepare(circ, True)
    c.set_plan_units(0)
    plan = c.region_plan(256)
    kinds = (plan["item"][:, 2].astype(np.int64) & 0xFFFFFFFF) >> 30
    assert (kinds != 2).all()
    assert len(plan["part_ptr"]) == 3 and int(plan["part_ptr"][-1]) == 2 * ((5000 + 31) // 32)
    assert len(plan["hfold"]) == int(plan["part_ptr"][-1])
    # the same chain cut for 32 compute units: the one-wave regions of the last round
    # hold 32 PMOS each, still whole parts
    c.set_plan_units(32)
    plan = c.region_plan(256)
    kinds = (plan["item"][:, 2].astype(np.int64) & 0xFFFFFFFF) >> 30
    assert (kinds != 2).all()
