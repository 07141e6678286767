"""Seeded synthetic circuit generators (inputs only; no model or stamping arithmetic).

Every workload of the method is a MOSFET netlist evaluated at one Newton-Raphson
operating point (Introduction: each NR iteration evaluates the device models at the
present operating point and forms the linearised MNA system).  The paper's own
netlists (the 28T full adder of Fig. "schematic", the Benchmark-1 instance sets) are
not published, so these generators stand in for them with the shapes named by the
workload definitions: inverter chains and rings (low conflict), a 6T SRAM array
(high conflict: bitlines and wordlines are shared nets), a 5T OTA (the colouring
example of Fig. "6tota-coloring") and two-stage op-amps for the batched sizing sweep.

Conventions shared by every generator
-------------------------------------
* node 0 is ground; node 1 is the supply rail ``vdd`` driven by one voltage source
  (vdd, ground) of value ``vdd``.
* ``term[k] = (d, g, s, b)`` node ids of device k; ``pol[k]`` is +1 (NMOS) or -1 (PMOS).
  NMOS bodies sit on ground, PMOS bodies on vdd.
* MNA rows: non-ground node n -> row n-1, then one branch row per voltage source.
* ``exclude`` marks the source-driven rail (vdd) so that callers can choose the
  rail-excluded conflict rule; ground is always non-conflicting.
* Random draws use ``numpy.random.Generator(PCG64(seed))`` in a fixed order per
  circuit: W, then L, then z ~ N(0,1) with VTH0 = 0.40*pol + 0.02*z, then x.
  ``x[vdd row] = vdd`` exactly and branch rows are 0.0; every other node voltage is
  U[0, vdd).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

NMOS = 1
PMOS = -1


@dataclasses.dataclass
class Circuit:
    name: str
    n_nodes: int                 # including ground node 0
    term: np.ndarray             # int32 (n_dev, 4): d, g, s, b
    pol: np.ndarray              # int8 (n_dev,)
    vsrc: np.ndarray             # int32 (n_vsrc, 2): pos, neg
    vsrc_volts: np.ndarray       # float64 (n_vsrc,)
    exclude: np.ndarray          # uint8 (n_nodes,): 1 = source-driven rail
    vdd: float
    W: np.ndarray | None = None  # float64 (n_dev,) metres
    L: np.ndarray | None = None
    VTH0: np.ndarray | None = None
    x: np.ndarray | None = None  # float64 (n_rows,)
    res: np.ndarray | None = None    # int32 (n_res, 2): series resistors' nodes (linear elements)
    res_g: np.ndarray | None = None  # float64 (n_res,): their conductances, siemens

    @property
    def n_res(self) -> int:
        return 0 if self.res is None else int(self.res.shape[0])

    @property
    def n_dev(self) -> int:
        return int(self.term.shape[0])

    @property
    def n_rows(self) -> int:
        return self.n_nodes - 1 + int(self.vsrc.shape[0])


def default_card(pol: int, symmetric: bool = False) -> dict:
    """Model-card values (SI units) for the BSIM4-core subset; NMOS and PMOS differ in U0 only.

    ``symmetric=True`` gives the PMOS card the NMOS mobility (used for the inverter
    transfer-point check)."""
    card = dict(
        tnom=300.15, toxe=1.8e-9, ndep=1.7e23, phis=0.85, vbi=1.0, k1=0.53, k2=-0.0186,
        k3=80.0, w0=2.5e-6, dvt0=1.0, dvt1=0.53, dsub=0.56, eta0=0.08, nfactor=1.0,
        cdsc=2.4e-4, voff=-0.08, u0=0.067, ua=1e-9, ub=1e-19, uc=-4.65e-11, vsat=8e4,
        a0=1.0, xj=1.5e-7, delta=0.01, delta1=1e-3, lambda_l=4.5e-9, cgdo=3e-10,
        lint=0.0, wint=0.0,
        # source/drain-body junctions, off unless jmod = 1 (BSIM4's JSS, NJS, CJS, PBS
        # default values, abrupt grading; junction area Weff * hdif; the diode is
        # continued by its tangent above vjmax)
        jmod=0.0, js=1e-4, nj=1.0, cj=5e-4, pb=1.0, fc=0.5, hdif=1e-7, vjmax=0.8)
    if pol == PMOS and not symmetric:
        card["u0"] = 0.025
    return card


def junction_card(pol: int, **over) -> dict:
    """The default card with the source/drain-body junctions on (the second model
    level behind the same kernels), optionally overriding junction parameters."""
    card = default_card(pol)
    card.update(jmod=1.0, **over)
    return card


CARD_FIELDS = ("tnom", "toxe", "ndep", "phis", "vbi", "k1", "k2", "k3", "w0", "dvt0", "dvt1",
               "dsub", "eta0", "nfactor", "cdsc", "voff", "u0", "ua", "ub", "uc", "vsat", "a0",
               "xj", "delta", "delta1", "lambda_l", "cgdo", "lint", "wint",
               "jmod", "js", "nj", "cj", "pb", "fc", "hdif", "vjmax")


def _finish(name, n_nodes, devs, vdd):
    term = np.array([d[0] for d in devs], dtype=np.int32).reshape(-1, 4)
    pol = np.array([d[1] for d in devs], dtype=np.int8)
    vsrc = np.array([[1, 0]], dtype=np.int32)
    excl = np.zeros(n_nodes, dtype=np.uint8)
    excl[1] = 1
    return Circuit(name, n_nodes, term, pol, vsrc, np.array([vdd], dtype=np.float64), excl, vdd)


def inverter_chain(n_stages: int, vdd: float = 1.0) -> Circuit:
    """Chain of CMOS inverters.  Nodes: 0 gnd, 1 vdd, 2 in, 3.. out_i.  Stage i: NMOS
    (out_i, in_i, gnd, gnd) then PMOS (out_i, in_i, vdd, vdd)."""
    devs = []
    for i in range(n_stages):
        inp = 2 if i == 0 else 3 + i - 1
        out = 3 + i
        devs.append(((out, inp, 0, 0), NMOS))
        devs.append(((out, inp, 1, 1), PMOS))
    return _finish(f"chain{n_stages}", 3 + n_stages, devs, vdd)


def inverter_chain_fast(n_stages: int, vdd: float = 1.0) -> Circuit:
    """Vectorised ``inverter_chain`` for large N (identical arrays)."""
    i = np.arange(n_stages, dtype=np.int64)
    out = 3 + i
    inp = np.where(i == 0, 2, 2 + i)
    term = np.zeros((2 * n_stages, 4), dtype=np.int32)
    term[0::2, 0] = out
    term[0::2, 1] = inp
    term[1::2, 0] = out
    term[1::2, 1] = inp
    term[1::2, 2] = 1
    term[1::2, 3] = 1
    pol = np.empty(2 * n_stages, dtype=np.int8)
    pol[0::2] = NMOS
    pol[1::2] = PMOS
    excl = np.zeros(3 + n_stages, dtype=np.uint8)
    excl[1] = 1
    return Circuit(f"chain{n_stages}", 3 + n_stages, term, pol, np.array([[1, 0]], np.int32),
                   np.array([vdd]), excl, vdd)


def parallel_chain(n_stages: int, group: int, vdd: float = 1.0) -> Circuit:
    """Chain whose stage i is ``group`` inverters in parallel sharing in_i and out_i
    (conflict-count sweep: adjacent stages form a clique of 4*group devices)."""
    i = np.repeat(np.arange(n_stages, dtype=np.int64), group)
    out = 3 + i
    inp = np.where(i == 0, 2, 2 + i)
    n = n_stages * group
    term = np.zeros((2 * n, 4), dtype=np.int32)
    term[0::2, 0] = out
    term[0::2, 1] = inp
    term[1::2, 0] = out
    term[1::2, 1] = inp
    term[1::2, 2] = 1
    term[1::2, 3] = 1
    pol = np.empty(2 * n, dtype=np.int8)
    pol[0::2] = NMOS
    pol[1::2] = PMOS
    excl = np.zeros(3 + n_stages, dtype=np.uint8)
    excl[1] = 1
    return Circuit(f"pchain{n_stages}x{group}", 3 + n_stages, term, pol,
                   np.array([[1, 0]], np.int32), np.array([vdd]), excl, vdd)


def ring_oscillator(n_stages: int, vdd: float = 1.0) -> Circuit:
    """Ring of ``n_stages`` inverters (odd).  Nodes: 0 gnd, 1 vdd, 2.. out_i; stage i
    takes out_{i-1} (stage 0 takes out_{n-1})."""
    i = np.arange(n_stages, dtype=np.int64)
    out = 2 + i
    inp = 2 + (i - 1) % n_stages
    term = np.zeros((2 * n_stages, 4), dtype=np.int32)
    term[0::2, 0] = out
    term[0::2, 1] = inp
    term[1::2, 0] = out
    term[1::2, 1] = inp
    term[1::2, 2] = 1
    term[1::2, 3] = 1
    pol = np.empty(2 * n_stages, dtype=np.int8)
    pol[0::2] = NMOS
    pol[1::2] = PMOS
    excl = np.zeros(2 + n_stages, dtype=np.uint8)
    excl[1] = 1
    return Circuit(f"ring{n_stages}", 2 + n_stages, term, pol, np.array([[1, 0]], np.int32),
                   np.array([vdd]), excl, vdd)


def sram6t(rows: int, cols: int, vdd: float = 1.0) -> Circuit:
    """6T SRAM array.  Nodes: 0 gnd, 1 vdd, WL_r, then (BL_c, BLB_c) pairs, then (Q, QB)
    per cell in row-major order.  Per cell: PU1 P(Q,QB,vdd,vdd), PD1 N(Q,QB,gnd,gnd),
    PU2 P(QB,Q,vdd,vdd), PD2 N(QB,Q,gnd,gnd), AX1 N(BL,WL,Q,gnd), AX2 N(BLB,WL,QB,gnd)."""
    r = np.repeat(np.arange(rows, dtype=np.int64), cols)
    c = np.tile(np.arange(cols, dtype=np.int64), rows)
    wl = 2 + r
    bl = 2 + rows + 2 * c
    blb = bl + 1
    q = 2 + rows + 2 * cols + 2 * (r * cols + c)
    qb = q + 1
    n = rows * cols
    term = np.zeros((6 * n, 4), dtype=np.int32)
    pol = np.empty(6 * n, dtype=np.int8)
    z = np.zeros_like(q)
    one = np.ones_like(q)
    cells = [((q, qb, one, one), PMOS), ((q, qb, z, z), NMOS), ((qb, q, one, one), PMOS),
             ((qb, q, z, z), NMOS), ((bl, wl, q, z), NMOS), ((blb, wl, qb, z), NMOS)]
    for j, (tt, p) in enumerate(cells):
        for t in range(4):
            term[j::6, t] = tt[t]
        pol[j::6] = p
    n_nodes = 2 + rows + 2 * cols + 2 * n
    excl = np.zeros(n_nodes, dtype=np.uint8)
    excl[1] = 1
    return Circuit(f"sram{rows}x{cols}", n_nodes, term, pol, np.array([[1, 0]], np.int32),
                   np.array([vdd]), excl, vdd)


def ota5t(vdd: float = 1.0) -> Circuit:
    """Five-transistor OTA with a current-mirror load (the colouring example of Fig.
    "6tota-coloring").  Nodes: 0 gnd, 1 vdd, 2 inp, 3 inn, 4 tail, 5 n1 (mirror), 6 out,
    7 bias.  M1 N(n1,inp,tail,gnd), M2 N(out,inn,tail,gnd), M3 P(n1,n1,vdd,vdd),
    M4 P(out,n1,vdd,vdd), M5 N(tail,bias,gnd,gnd)."""
    devs = [((5, 2, 4, 0), NMOS), ((6, 3, 4, 0), NMOS), ((5, 5, 1, 1), PMOS),
            ((6, 5, 1, 1), PMOS), ((4, 7, 0, 0), NMOS)]
    return _finish("ota5t", 8, devs, vdd)


def opamp2(n_fet: int, vdd: float = 1.0) -> Circuit:
    """Two-stage op-amp with ``n_fet`` in 8..14 transistors.  Nodes: 0 gnd, 1 vdd,
    2 inp, 3 inn, 4 tail, 5 n1, 6 out1, 7 out, 8 bias, 9.. series-diode nodes.
    Core: M1 N(n1,inp,tail,gnd), M2 N(out1,inn,tail,gnd), M3 P(n1,n1,vdd,vdd),
    M4 P(out1,n1,vdd,vdd), M5 N(tail,bias,gnd,gnd), M6 P(out,out1,vdd,vdd),
    M7 N(out,bias,gnd,gnd), M8 N(bias,bias,gnd,gnd); then n_fet-8 diode-connected PMOS
    in series from vdd down into the bias node (bodies on vdd)."""
    assert 8 <= n_fet <= 14
    devs = [((5, 2, 4, 0), NMOS), ((6, 3, 4, 0), NMOS), ((5, 5, 1, 1), PMOS),
            ((6, 5, 1, 1), PMOS), ((4, 8, 0, 0), NMOS), ((7, 6, 1, 1), PMOS),
            ((7, 8, 0, 0), NMOS), ((8, 8, 0, 0), NMOS)]
    m = n_fet - 8
    n_nodes = 9 + max(m - 1, 0)
    prev = 1
    for j in range(m):
        nxt = 8 if j == m - 1 else 9 + j
        devs.append(((nxt, nxt, prev, 1), PMOS))
        prev = nxt
    return _finish(f"opamp{n_fet}", n_nodes, devs, vdd)


def ripple_adder28(n_bits: int, vdd: float = 1.0) -> Circuit:
    """Ripple-carry adder of ``n_bits`` 28-transistor mirror full adders (14 PMOS, 14
    NMOS per bit), the cell shape of the paper's 64-bit adder benchmark (Fig.
    "schematic", Table I: 1,792 FETs for 64 bits).  Nodes: 0 gnd, 1 vdd, 2 c0, then per
    bit i sixteen nodes: a, b, cob, x1, x2, y1, y2, sb, x3, x4, x5, y3, y4, y5, s, co
    (co is the next bit's carry in c).  Per bit, the pull-up devices first:
      P(y1,a,vdd) P(cob,b,y1) P(y2,a,vdd) P(y2,b,vdd) P(cob,c,y2)       carry mirror
      P(y3,a,vdd) P(y4,b,y3) P(sb,c,y4) P(y5,a,vdd) P(y5,b,vdd) P(y5,c,vdd) P(sb,cob,y5)
      P(s,sb,vdd) P(co,cob,vdd)                                          inverters
    then the pull-down devices:
      N(cob,a,x1) N(x1,b,gnd) N(cob,c,x2) N(x2,a,gnd) N(x2,b,gnd)        cob = not(ab + c(a+b))
      N(sb,a,x3) N(x3,b,x4) N(x4,c,gnd) N(sb,cob,x5) N(x5,a,gnd) N(x5,b,gnd) N(x5,c,gnd)
                                                            sb = not(abc + cob(a+b+c))
      N(s,sb,gnd) N(co,cob,gnd)                                          s, co
    Bodies: NMOS on ground, PMOS on vdd.  With this listing the greedy colouring under
    the paper's rule (only ground excluded) needs exactly one colour per PMOS, 14 per
    bit (every PMOS body is on vdd), the 896 of Table I for 64 bits."""
    devs = []
    c = 2
    for i in range(n_bits):
        base = 3 + 16 * i
        a, b, cob, x1, x2, y1, y2, sb, x3, x4, x5, y3, y4, y5, sn, co = range(base, base + 16)
        N = lambda d, g, s_: devs.append(((d, g, s_, 0), NMOS))
        P = lambda d, g, s_: devs.append(((d, g, s_, 1), PMOS))
        P(y1, a, 1); P(cob, b, y1); P(y2, a, 1); P(y2, b, 1); P(cob, c, y2)
        P(y3, a, 1); P(y4, b, y3); P(sb, c, y4); P(y5, a, 1); P(y5, b, 1); P(y5, c, 1); P(sb, cob, y5)
        P(sn, sb, 1); P(co, cob, 1)
        N(cob, a, x1); N(x1, b, 0); N(cob, c, x2); N(x2, a, 0); N(x2, b, 0)
        N(sb, a, x3); N(x3, b, x4); N(x4, c, 0); N(sb, cob, x5); N(x5, a, 0); N(x5, b, 0); N(x5, c, 0)
        N(sn, sb, 0); N(co, cob, 0)
        c = co
    return _finish(f"adder{n_bits}x28", 3 + 16 * n_bits, devs, vdd)


R_SERIES = 1e-3   # ohm: the series resistors of Table I's R14 and R89 netlists


def split_nets(circ: Circuit, rule: str) -> tuple[Circuit, int]:
    """Series-resistor net splitting (Table I's R rows): chosen terminal connections
    of each FET move to a private node, tied back to the original net by a series
    resistor of R_SERIES.  Returns the netlist (private nodes appended after the
    original ones, in device then terminal order; resistor j joins private node and
    original net, in that order, with conductance 1/R_SERIES) and the number of
    resistors.  The resistors are linear elements stamped after the FETs; the FET
    conflict graph only sees that the FETs no longer share those nets.
      rule "all":  every non-ground terminal connection (no two FETs share a node)
      rule "rail": the vdd connections of each FET (its vdd-tied terminals share one
                   private node per FET)"""
    term = circ.term.copy()
    n_nodes = circ.n_nodes
    res = []
    for k in range(circ.n_dev):
        if rule == "all":
            for t in range(4):
                if term[k, t] != 0:
                    res.append((n_nodes, int(circ.term[k, t])))
                    term[k, t] = n_nodes
                    n_nodes += 1
        elif rule == "rail":
            on = [t for t in range(4) if circ.term[k, t] == 1]
            if on:
                res.append((n_nodes, 1))
                term[k, on] = n_nodes
                n_nodes += 1
        else:
            raise ValueError(rule)
    excl = np.zeros(n_nodes, dtype=np.uint8)
    excl[:circ.n_nodes] = circ.exclude
    r = np.array(res, dtype=np.int32).reshape(-1, 2)
    g = np.full(r.shape[0], 1.0 / R_SERIES)
    return Circuit(f"{circ.name}_{rule}", n_nodes, term, circ.pol.copy(), circ.vsrc.copy(),
                   circ.vsrc_volts.copy(), excl, circ.vdd, res=r, res_g=g), r.shape[0]


def with_random_resistors(circ: Circuit, n_res: int, seed: int) -> Circuit:
    """Add resistors between uniformly drawn nodes (ground, vdd, self-loops and
    parallel pairs included) with conductances uniform in [1e-4, 1e-2] S: linear
    parts on entries the FETs also write, on rail entries and on new entries."""
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.integers(0, circ.n_nodes, size=(n_res, 2)).astype(np.int32)
    g = rng.uniform(1e-4, 1e-2, n_res)
    if circ.res is not None:
        r = np.concatenate([circ.res, r])
        g = np.concatenate([circ.res_g, g])
    circ.res, circ.res_g = r, g
    return circ


def adder_case(n_bits: int, seed: int, split: str | None = None) -> Circuit:
    rng = np.random.Generator(np.random.PCG64(seed))
    c = ripple_adder28(n_bits)
    if split:
        c, _ = split_nets(c, split)
    return draw_params(c, rng, W_CHAIN, L_CHAIN)


def random_netlist(n_dev: int, n_nodes: int, seed: int, vdd: float = 1.0) -> Circuit:
    """FETs whose four terminals are drawn uniformly from nodes 0..n_nodes-1 (0
    ground, 1 vdd), polarity at random; with few nodes every coincidence pattern of
    the terminals occurs.  The first devices are degenerate on purpose: all four
    terminals on ground, drain and source on one node, every terminal on vdd."""
    rng = np.random.Generator(np.random.PCG64(seed))
    term = rng.integers(0, n_nodes, size=(n_dev, 4)).astype(np.int32)
    pol = np.where(rng.random(n_dev) < 0.5, NMOS, PMOS).astype(np.int8)
    special = [(0, 0, 0, 0), (2, 3, 2, 0), (1, 1, 1, 1), (2, 2, 2, 2), (3, 0, 3, 3)]
    for i, t in enumerate(special[:n_dev]):
        term[i] = t
    excl = np.zeros(n_nodes, dtype=np.uint8)
    excl[1] = 1
    return Circuit(f"random{n_dev}x{n_nodes}", n_nodes, term, pol, np.array([[1, 0]], np.int32),
                   np.array([vdd]), excl, vdd)


def no_shared_nets(n_dev: int, vdd: float = 1.0) -> Circuit:
    """Devices whose terminals all sit on private nodes or ground (every net split,
    as by the series-resistor transform of Benchmark 2): the conflict graph is empty."""
    term = np.zeros((n_dev, 4), dtype=np.int32)
    base = 2 + 2 * np.arange(n_dev, dtype=np.int64)
    term[:, 0] = base
    term[:, 1] = base + 1
    pol = np.full(n_dev, NMOS, dtype=np.int8)
    excl = np.zeros(2 + 2 * n_dev, dtype=np.uint8)
    excl[1] = 1
    return Circuit(f"private{n_dev}", 2 + 2 * n_dev, term, pol, np.array([[1, 0]], np.int32),
                   np.array([vdd]), excl, vdd)


def draw_params(circ: Circuit, rng: np.random.Generator, w_range, l_range) -> Circuit:
    """W ~ U(w_range), L ~ U(l_range), VTH0 = 0.40*pol + 0.02*N(0,1), then x (see module doc)."""
    n = circ.n_dev
    circ.W = rng.uniform(w_range[0], w_range[1], n)
    circ.L = rng.uniform(l_range[0], l_range[1], n)
    z = rng.standard_normal(n)
    circ.VTH0 = 0.40 * circ.pol.astype(np.float64) + 0.02 * z
    x = rng.uniform(0.0, circ.vdd, circ.n_rows)
    x[0] = circ.vdd                       # row of node 1 (vdd)
    x[circ.n_nodes - 1:] = 0.0            # branch rows
    circ.x = x
    return circ


W_CHAIN = (0.2e-6, 2.0e-6)
L_CHAIN = (45e-9, 90e-9)
W_SRAM = (0.1e-6, 0.3e-6)
L_SRAM = (45e-9, 45e-9)
W_OPAMP = (0.5e-6, 20e-6)
L_OPAMP = (45e-9, 500e-9)


def chain_case(n_stages: int, seed: int) -> Circuit:
    rng = np.random.Generator(np.random.PCG64(seed))
    c = inverter_chain_fast(n_stages) if n_stages > 64 else inverter_chain(n_stages)
    return draw_params(c, rng, W_CHAIN, L_CHAIN)


def drive(circ: Circuit, node: int, volts: float) -> Circuit:
    """Hold `node` at `volts` with one more voltage source to ground (its branch row
    follows the existing ones).  Before ``draw_params``, which sizes x."""
    circ.vsrc = np.concatenate([circ.vsrc, np.array([[node, 0]], np.int32)])
    circ.vsrc_volts = np.concatenate([circ.vsrc_volts, [float(volts)]])
    return circ


def chain_dc_case(n_stages: int, seed: int, vin: float = 0.0) -> Circuit:
    """Inverter chain with its input (node 2) held at `vin`: a circuit with a unique
    DC operating point (every node has a conductive path; gates are driven)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    c = inverter_chain_fast(n_stages) if n_stages > 64 else inverter_chain(n_stages)
    return draw_params(drive(c, 2, vin), rng, W_CHAIN, L_CHAIN)


def pchain_case(n_dev: int, group: int, seed: int) -> Circuit:
    """Parallel-inverter chain of about ``n_dev`` devices, ``group`` inverters per stage
    (at least two stages), chain parameter ranges."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return draw_params(parallel_chain(max(2, n_dev // (2 * group)), group), rng, W_CHAIN, L_CHAIN)


def sram_case(rows: int, cols: int, seed: int) -> Circuit:
    rng = np.random.Generator(np.random.PCG64(seed))
    return draw_params(sram6t(rows, cols), rng, W_SRAM, L_SRAM)


def workload(idx: int) -> Circuit | list:
    """The five workloads: 0 chain 50, 1 chain 100000, 2 SRAM 256x256, 3 batch of 512,
    4 chain 10000 (the differentiation case; its batch half is ``workload(3)``)."""
    if idx == 0:
        return chain_case(50, seed=1)
    if idx == 1:
        return chain_case(100_000, seed=2)
    if idx == 2:
        return sram_case(256, 256, seed=3)
    if idx == 3:
        return batch_sweep(seed=4)
    if idx == 4:
        return chain_case(10_000, seed=5)
    raise ValueError(idx)


def _log_uniform_int(rng, lo, hi, odd=False):
    v = math.exp(rng.uniform(math.log(lo), math.log(hi)))
    if odd:
        k = int(round((v - 1.0) / 2.0)) * 2 + 1
        return min(max(k, lo if lo % 2 else lo + 1), hi if hi % 2 else hi - 1)
    return min(max(int(round(v)), lo), hi)


def batch_sweep(seed: int = 4, n_opamp: int = 256, n_chain: int = 192, n_ring: int = 64,
                chain_range=(100, 10_000), ring_range=(501, 50_001)) -> list:
    """Sizing-sweep batch: op-amps (8..14 FETs), chains (log-uniform stages), odd rings
    (log-uniform stages); order shuffled by the seed.  Per circuit, in batch order:
    vdd ~ U[0.8, 1.2], then W, L, z, x as in ``draw_params``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    plan = []
    for _ in range(n_opamp):
        plan.append(("opamp", int(rng.integers(8, 15))))
    for _ in range(n_chain):
        plan.append(("chain", _log_uniform_int(rng, *chain_range)))
    for _ in range(n_ring):
        plan.append(("ring", _log_uniform_int(rng, *ring_range, odd=True)))
    order = rng.permutation(len(plan))
    out = []
    for k in order:
        kind, size = plan[k]
        vdd = float(rng.uniform(0.8, 1.2))
        if kind == "opamp":
            c = draw_params(opamp2(size, vdd), rng, W_OPAMP, L_OPAMP)
        elif kind == "chain":
            c = draw_params(inverter_chain_fast(size, vdd), rng, W_CHAIN, L_CHAIN)
        else:
            c = draw_params(ring_oscillator(size, vdd), rng, W_CHAIN, L_CHAIN)
        out.append(c)
    return out


def cotangents(n_nnz: int, n_rows: int, seed: int = 50):
    """Cotangents on A's nonzeros and on b, both N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(n_nnz), rng.standard_normal(n_rows)
