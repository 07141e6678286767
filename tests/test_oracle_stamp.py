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
  where the chunk shape decides the result."""
import numpy as np
import pytest

from paper_2604_03079_amd import netgen as G

NC, PC = G.default_card(1), G.default_card(-1)


def residual(orc, circ, x, ag0, hist=None):
    F = np.zeros(circ.n_rows)
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


@pytest.mark.parametrize("make", [lambda: G.workload(0), lambda: G.draw_params(
    G.opamp2(12), np.random.default_rng(3), G.W_OPAMP, G.L_OPAMP), lambda: G.sram_case(3, 4, 9)],
    ids=["chain50", "opamp12", "sram3x4"])
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
    # chunk 0 = [2^53, 1 x 255]: a left fold loses every 1 (ties to even);
    # chunk 1 = [1 x 256] sums to 256 exactly; the hub sum adds the chunk sums.
    c = np.ones(512)
    c[0] = 2.0 ** 53
    assert orc.hubsum(c) == 2.0 ** 53 + 256
    assert orc.hubsum(c[:256]) == 2.0 ** 53                  # m <= 256: plain fold
    d = np.cumsum(c[:200])                                    # sequential fold
    assert orc.hubsum(c[:200]) == d[-1]
    # three levels (m > 256^2): integers add exactly whatever the shape
    big = np.arange(70_000, dtype=np.float64)
    assert orc.hubsum(big) == float(big.sum())
    rng = np.random.default_rng(1)
    r = rng.standard_normal(100_000)
    import math
    assert abs(orc.hubsum(r) - math.fsum(r)) <= 1e-13 * np.abs(r).sum()


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
    s = vals[0]
    for x in vals[1:]:
        s = s + x
    assert A[rp[0]] == s          # (vdd, vdd) is the first entry of row 0
