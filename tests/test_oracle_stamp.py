"""Pins of the oracle's stamp phase (Methodology: per-instance contributions are
accumulated into the global MNA matrix A and right-hand side b).

* The assembled system reproduces Newton's linearisation at x: on node rows
  A x - b equals the circuit residual F(x) = sum over devices of I + ag0*Q - hist,
  computed here from per-device currents and charges only, and A is the
  finite-difference Jacobian of F (plus the source stamps).
* Colour replay (colours in sequence, first writer stores) and serial order give
  the same sums up to reordering: per entry within 1e-12 of the sum of
  |contributions|.  Replay is bitwise repeatable.
* The fixed-shape hub sum (chunks of 256, then recursively) is pinned by a case
  where the chunk shape decides the result.
* Series resistors of a split netlist (Benchmark 2, Table I's R rows): their linear
  part is the incidence-matrix Laplacian N diag(g) N^T; a resistor divider solved
  from the assembled system gives the closed-form divider voltages; merging every
  private node back onto its original net gives the unsplit circuit's system; and
  the split system is Newton's linearisation of KCL with resistor currents."""
import numpy as np
import pytest

from paper_2604_03079_amd import netgen as G

NC, PC = G.default_card(1), G.default_card(-1)


def residual(orc, circ, x, ag0, hist=None):
    F = np.zeros(circ.n_rows)
    for (p, q), g in zip(circ.res if circ.res is not None else [], circ.res_g if circ.res is not None else []):
        i = g * ((0.0 if p == 0 else x[p - 1]) - (0.0 if q == 0 else x[q - 1]))   # p -> q
        if p:
            F[p - 1] += i
        if q:
            F[q - 1] -= i
    for v in range(circ.n_dev):
        t = circ.term[v]
        V = np.array([0.0 if n == 0 else x[n - 1] for n in t])
        _, _, I, Q = orc.device_eval(NC if circ.pol[v] > 0 else PC, int(circ.pol[v]), circ.W[v],
                                     circ.L[v], circ.VTH0[v], V, ag0,
                                     None if hist is None else hist[v])
        for k in range(4):
            if t[k] != 0:
                F[t[k] - 1] += I[k] + ag0 * Q[k] - (0.0 if hist is None else hist[v][k])
    return F


def dense(rp, ci, A, n):
    M = np.zeros((n, n))
    for r in range(n):
        M[r, ci[rp[r]:rp[r + 1]]] = A[rp[r]:rp[r + 1]]
    return M


def split_case(rule, seed):
    # a one-bit adder cell split by series resistors whose conductances are drawn so
    # that resistor and FET currents are of one order
    circ, _ = G.split_nets(G.ripple_adder28(1), rule)
    circ = G.draw_params(circ, np.random.default_rng(seed), G.W_CHAIN, G.L_CHAIN)
    circ.res_g = np.random.default_rng(seed + 1).uniform(1e-5, 1e-3, circ.n_res)
    return circ


@pytest.mark.parametrize("make", [lambda: G.workload(0), lambda: G.draw_params(
    G.opamp2(12), np.random.default_rng(3), G.W_OPAMP, G.L_OPAMP), lambda: G.sram_case(3, 4, 9),
    lambda: split_case("all", 5), lambda: split_case("rail", 6)],
    ids=["chain50", "opamp12", "sram3x4", "adder1r89", "adder1r14"])
def test_assembly_is_newtons_linearisation(orc, make):
    circ = make()
    rng = np.random.default_rng(0)
    hist = rng.normal(0, 1e-5, (circ.n_dev, 4))
    ag0 = 1e12
    rp, ci = orc.pattern(circ)
    A, b = orc.assemble(circ, rp, ci, NC, PC, ag0, hist)
    n_node = circ.n_nodes - 1
    M = dense(rp, ci, A, circ.n_rows)
    F = residual(orc, circ, circ.x, ag0, hist)
    r = M @ circ.x - b
    scale = np.abs(M[:n_node]).max() * np.abs(circ.x).max()
    assert np.allclose(r[:n_node], F[:n_node], rtol=0, atol=1e-12 * scale)
    # source rows: branch equation x[vdd] - Vdd = 0 and the branch column
    br = n_node
    assert M[br, 0] == 1.0 and M[0, br] == 1.0 and b[br] == circ.vdd and r[br] == 0.0
    # A is the Jacobian of F (node rows/cols)
    eps = 1e-7
    for j in range(n_node):
        xp = circ.x.copy(); xp[j] += eps
        xm = circ.x.copy(); xm[j] -= eps
        col = (residual(orc, circ, xp, ag0, hist) - residual(orc, circ, xm, ag0, hist)) / (2 * eps)
        assert np.allclose(col[:n_node], M[:n_node, j], rtol=0, atol=1e-6 * np.abs(M).max())


@pytest.mark.parametrize("idx", [0, 1])
def test_replay_matches_serial_within_reordering_bound(orc, idx):
    circ = G.workload(idx)
    rp, ci = orc.pattern(circ)
    for exclude in (True, False) if idx == 0 else (True,):
        col, C, _ = orc.colour(circ, exclude)
        A1, b1 = orc.assemble(circ, rp, ci, NC, PC, 1e12, col=col, exclude=exclude)
        A2, b2 = orc.assemble(circ, rp, ci, NC, PC, 1e12, col=col, exclude=exclude)
        assert np.array_equal(A1.view(np.int64), A2.view(np.int64))
        assert np.array_equal(b1.view(np.int64), b2.view(np.int64))
        As, bs = orc.assemble(circ, rp, ci, NC, PC, 1e12)
        mA, mb = orc.assemble_magnitude(circ, rp, ci, NC, PC, 1e12)
        assert np.all(np.abs(A1 - As) <= 1e-12 * mA)
        assert np.all(np.abs(b1 - bs) <= 1e-12 * mb)


def test_hubsum_shape(orc):
    # The hub sum is the pairwise tree split at the largest power of two below m.
    # Values are hand-derived from binary64 round-to-nearest-even: 2^53 + 1 rounds
    # to 2^53 (a tie), 2^53 + 2k is exact for small k.
    t53 = 2.0 ** 53
    # (c0 + c1) + (c2 + c3): the first 1 is lost, the pair (1 + 1) is not; a left fold
    # would lose all three
    assert orc.hubsum([t53, 1.0, 1.0, 1.0]) == t53 + 2
    # m = 3 splits as (c0 + c1) + c2 (both ones lost), not c0 + (c1 + c2) (= 2^53 + 2)
    assert orc.hubsum([t53, 1.0, 1.0]) == t53
    assert orc.hubsum([1.0, 1.0, t53]) == t53 + 2          # (1 + 1) + 2^53
    # m = 6 splits at 4: (1 + 1) + (1 + 1) = 4, then (2^53 + 1) + 1 -> 2^53, sum 2^53 + 4;
    # a split at 3 would give ((1 + 1) + 1) + ((1 + 2^53) + 1) = 3 + 2^53 -> 2^53 + 4
    # as well, so the next case separates them
    assert orc.hubsum([1.0, 1.0, 1.0, 1.0, t53, 1.0]) == t53 + 4
    # m = 6, [2^53, 1, 1, 1, 1, 1]: split at 4 gives (2^53 + 2) + (1 + 1) = 2^53 + 4;
    # a split at 3 gives (2^53 + 1 -> 2^53, + 1 -> 2^53) + 3 -> 2^53 + 4 (tie to even
    # of 2^53 + 3 is 2^53 + 4) -- equal again; a left fold gives 2^53
    assert orc.hubsum([t53] + [1.0] * 5) == t53 + 4
    # 2^53 followed by 255 ones: every aligned block of 2^j ones sums exactly to 2^j,
    # and the block holding 2^53 grows 2^53, 2^53 + 2, + 4, ..., + 128: 2^53 + 254
    c = np.ones(512)
    c[0] = t53
    assert orc.hubsum(c[:256]) == t53 + 254
    assert orc.hubsum(c) == t53 + 254 + 256
    # 1 followed by 2^16 - 1 copies of 2^-53: only the first tiny value is lost (1 +
    # 2^-53 is a tie), every later block of tiny values arrives as a multiple of
    # 2^-52 and is exact: 1 + (2^15 - 1) 2^-52; a left fold returns 1
    tiny = np.full(2 ** 16, 2.0 ** -53)
    tiny[0] = 1.0
    assert orc.hubsum(tiny) == 1.0 + (2 ** 15 - 1) * 2.0 ** -52
    # -0.0 padding: a single -0.0, and -0.0 next to +0.0, keep IEEE signs
    assert np.signbit(orc.hubsum([-0.0]))
    assert not np.signbit(orc.hubsum([-0.0, 0.0, -0.0]))
    # integers add exactly whatever the shape (no contribution dropped or repeated)
    big = np.arange(70_000, dtype=np.float64)
    assert orc.hubsum(big) == float(big.sum())
    # the pairwise error bound: |sum - exact| <= ceil(log2 m) u sum |c|
    rng = np.random.default_rng(1)
    r = rng.standard_normal(100_000)
    import math
    assert abs(orc.hubsum(r) - math.fsum(r)) <= 17 * 2.0 ** -53 * np.abs(r).sum()


def test_replay_uses_hubsum_for_rail_entries(orc):
    circ = G.workload(0)
    rp, ci = orc.pattern(circ)
    col, C, _ = orc.colour(circ, True)
    A, b = orc.assemble(circ, rp, ci, NC, PC, 1e12, col=col, exclude=True)
    slot, sflag, brow, bflag = orc.stamp_map(circ, rp, ci, col, True)
    # rebuild the (vdd, vdd) entry: merged PMOS contributions in ascending device order
    vals = []
    for v in range(circ.n_dev):
        if circ.pol[v] < 0:
            Y, bl, _, _ = orc.device_eval(PC, -1, circ.W[v], circ.L[v], circ.VTH0[v],
                                          [circ.x[circ.term[v][0] - 1], circ.x[circ.term[v][1] - 1],
                                           circ.vdd, circ.vdd], 1e12)
            vals.append(((Y[2, 2] + Y[2, 3]) + Y[3, 2]) + Y[3, 3])
    # 50 PMOS: the pairwise tree of 64 leaves, the last 14 being -0.0 padding; its
    # value lies within the pairwise bound of the exact sum, and the replayed entry
    # is that value (every PMOS contribution enters, in ascending device order)
    import math
    assert len(vals) == 50
    assert A[rp[0]] == orc.hubsum(vals)          # (vdd, vdd) is the first entry of row 0
    assert abs(A[rp[0]] - math.fsum(vals)) <= 6 * 2.0 ** -53 * sum(abs(v) for v in vals)
    assert A[rp[0]] == orc.hubsum(vals + [-0.0] * 14)


def netlist(n_nodes, res, g, term=None, pol=None, vdd=1.0):
    """A circuit of series resistors (and optional FETs) with vdd on node 1."""
    term = np.zeros((0, 4), np.int32) if term is None else np.asarray(term, np.int32).reshape(-1, 4)
    pol = np.zeros(0, np.int8) if pol is None else np.asarray(pol, np.int8)
    excl = np.zeros(n_nodes, np.uint8)
    c = G.Circuit("resnet", n_nodes, term, pol, np.array([[1, 0]], np.int32), np.array([vdd]), excl,
                  vdd, res=np.asarray(res, np.int32).reshape(-1, 2), res_g=np.asarray(g, np.float64))
    c.W = np.full(c.n_dev, 1e-6); c.L = np.full(c.n_dev, 50e-9); c.VTH0 = 0.4 * c.pol.astype(float)
    c.x = np.zeros(c.n_rows)
    return c


def test_linear_part_is_the_incidence_laplacian(orc):
    # dyadic conductances add exactly in any order, so the stamp sums must equal the
    # product N diag(g) N^T of the node-resistor incidence matrix bit for bit;
    # grounded resistors, parallel resistors and a self-loop (no effect) included
    rng = np.random.default_rng(11)
    n_nodes, m = 40, 300
    res = rng.integers(0, n_nodes, (m, 2)).astype(np.int32)
    res[:5] = [(3, 0), (0, 7), (5, 5), (9, 12), (12, 9)]
    g = rng.integers(1, 64, m) / 8.0
    circ = netlist(n_nodes, res, g)
    rp, ci = orc.pattern(circ)
    Lin, touched = orc.linear_stamp(circ, rp, ci)
    N = np.zeros((n_nodes, m))
    N[res[:, 0], np.arange(m)] += 1.0
    N[res[:, 1], np.arange(m)] -= 1.0
    lap = (N * g) @ N.T
    n = circ.n_rows
    D = dense(rp, ci, Lin, n)
    assert np.array_equal(D[:n_nodes - 1, :n_nodes - 1], lap[1:, 1:])
    assert not D[n_nodes - 1:].any() and not D[:, n_nodes - 1:].any()   # branch row untouched
    # touched: exactly the entries of non-ground resistor ends (self-loop's diagonal too)
    want = np.zeros((n, n), bool)
    for (p, q) in res:
        for r, c in ((p, p), (p, q), (q, p), (q, q)):
            if r and c:
                want[r - 1, c - 1] = True
    assert np.array_equal(dense(rp, ci, touched.astype(float), n) > 0, want)
    # magnitude: sum of |stamps|, the same product with the unsigned incidence matrix
    Lm, _ = orc.linear_stamp(circ, rp, ci, magnitude=True)
    U = np.zeros((n_nodes, m))
    U[res[:, 0], np.arange(m)] += 1.0
    U[res[:, 1], np.arange(m)] += 1.0
    lm = (U * g) @ U.T
    assert np.array_equal(dense(rp, ci, Lm, n)[:n_nodes - 1, :n_nodes - 1], lm[1:, 1:])


def test_resistor_divider_closed_form(orc):
    # vdd -> R0 -> node 2 -> R1 -> ... -> R_{k-1} -> ground: node j carries
    # Vdd * (sum of the resistances below it) / (total), the source carries Vdd / total
    R = np.array([1.0, 2.0, 3.0, 5.0, 8.0, 13.0])
    k = R.size
    nodes = [1] + list(range(2, k + 1)) + [0]
    res = [(nodes[i], nodes[i + 1]) for i in range(k)]
    vdd = 1.8
    circ = netlist(k + 1, res, 1.0 / R, vdd=vdd)
    rp, ci = orc.pattern(circ)
    for col in (None, np.zeros(0, np.int32)):
        A, b = orc.assemble(circ, rp, ci, NC, PC, 1e12, col=col)
        x = np.linalg.solve(dense(rp, ci, A, circ.n_rows), b)
        below = np.cumsum(R[::-1])[::-1]          # resistance from each node down to ground
        assert np.allclose(x[:k], vdd * below / R.sum(), rtol=1e-14, atol=0)
        assert np.isclose(x[k], -vdd / R.sum(), rtol=1e-14)   # branch current: into pos, out of neg


@pytest.mark.parametrize("rule", ["all", "rail"])
@pytest.mark.parametrize("make", [lambda: G.ripple_adder28(2), lambda: G.random_netlist(120, 9, 3),
                                  lambda: G.workload(0)], ids=["adder2", "random120x9", "chain50"])
def test_split_netlist_merges_back_onto_the_unsplit_system(orc, rule, make):
    # folding every private node back onto the net its resistor ties it to, with the
    # private nodes at their net's voltage, cancels the resistor stamps and leaves the
    # unsplit circuit's A and b (up to the reordering of the sums)
    base = make()
    if base.W is None:
        base = G.draw_params(base, np.random.default_rng(4), G.W_CHAIN, G.L_CHAIN)
    split, n_res = G.split_nets(base, rule)
    assert n_res == split.n_res > 0
    owner = np.arange(split.n_nodes)
    for p, q in split.res:
        owner[p] = q                               # private node -> original net
    assert np.all(owner[owner] == owner)
    n0, n1 = base.n_nodes - 1, split.n_nodes - 1
    rowmap = np.concatenate([owner[1:] - 1, n0 + np.arange(base.vsrc.shape[0])])
    split.W, split.L, split.VTH0 = base.W, base.L, base.VTH0
    split.x = base.x[rowmap]
    rp, ci = orc.pattern(base)
    A0, b0 = orc.assemble(base, rp, ci, NC, PC, 1e12)
    mA0, mb0 = orc.assemble_magnitude(base, rp, ci, NC, PC, 1e12)
    srp, sci = orc.pattern(split)
    for col in (None, orc.colour(split, False)[0]):
        A1, b1 = orc.assemble(split, srp, sci, NC, PC, 1e12, col=col)
        mA1, _ = orc.assemble_magnitude(split, srp, sci, NC, PC, 1e12)
        P = np.zeros((split.n_rows, base.n_rows))
        P[np.arange(split.n_rows), rowmap] = 1.0
        M = P.T @ dense(srp, sci, A1, split.n_rows) @ P
        Mm = P.T @ dense(srp, sci, mA1, split.n_rows) @ P
        assert np.all(np.abs(M - dense(rp, ci, A0, base.n_rows)) <= 1e-13 * (Mm + dense(rp, ci, mA0, base.n_rows)))
        assert np.all(np.abs(P.T @ b1 - b0) <= 1e-13 * mb0)
    # the split netlist's FETs share no net that the rule split
    if rule == "all":
        assert orc.colour(split, False)[1] == 1
