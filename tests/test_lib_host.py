"""CPU checks of the C-ABI library: it loads, exports every entry point declared in
include/colorstamp.h, its host setup (colouring, CSR pattern, stamp map) equals the
oracle's bit for bit, and argument/state errors are reported before any launch."""
import itertools
import os
import re

import numpy as np
import pytest

from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_entry_point():
    L = CS.lib()
    header = open(os.path.join(ROOT, "include", "colorstamp.h")).read()
    declared = set(re.findall(r"\b(cs_[a-z_]+)\s*\(", header))
    assert declared == set(CS.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


CASES = [
    ("chain50", lambda: G.workload(0)),
    ("ota5t", G.ota5t),
    ("opamp8", lambda: G.opamp2(8)),
    ("opamp14", lambda: G.opamp2(14)),
    ("ring11", lambda: G.ring_oscillator(11)),
    ("sram5x7", lambda: G.sram6t(5, 7)),
    ("pchain9x4", lambda: G.parallel_chain(9, 4)),
    ("private13", lambda: G.no_shared_nets(13)),
    ("chain1", lambda: G.inverter_chain(1)),
    ("adder3x28", lambda: G.ripple_adder28(3)),
    ("random600x6", lambda: G.random_netlist(600, 6, 21)),
    ("random2000x1500", lambda: G.random_netlist(2000, 1500, 22)),
    ("adder2r89", lambda: G.split_nets(G.ripple_adder28(2), "all")[0]),
    ("adder2r14", lambda: G.split_nets(G.ripple_adder28(2), "rail")[0]),
    ("random300x7r", lambda: G.split_nets(G.random_netlist(300, 7, 23), "all")[0]),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("exclude", [False, True])
def test_setup_equals_oracle(orc, name, make, exclude):
    circ = make()
    c = CS.Circuit.from_netlist(circ)
    col, C, E = c.colour(circ.exclude if exclude else None)
    ocol, oC, oE = orc.colour(circ, exclude)
    assert np.array_equal(col, ocol) and C == oC and E == oE
    c.build_map()
    rp, ci = c.pattern()
    orp, oci = orc.pattern(circ)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    for a, b in zip(c.stamp_map(), orc.stamp_map(circ, orp, oci, ocol, exclude)):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("exclude", [False, True])
@pytest.mark.parametrize("order", ["largest_first", "dsatur"])
def test_ordered_colouring_and_map_equal_oracle(orc, name, make, exclude, order):
    # the colouring in another vertex order, and the stamp map built on it
    circ = make()
    c = CS.Circuit.from_netlist(circ)
    col, C, E = c.colour(circ.exclude if exclude else None, order)
    ocol, oC, oE = orc.colour_order(circ, exclude, order)
    assert np.array_equal(col, ocol) and C == oC and E == oE
    c.build_map()
    orp, oci = orc.pattern(circ)
    for a, b in zip(c.stamp_map(), orc.stamp_map(circ, orp, oci, ocol, exclude)):
        assert np.array_equal(a, b)


def test_unknown_colouring_order_is_refused():
    c = CS.Circuit.from_netlist(G.workload(0))
    assert CS.lib().cs_build_coloring_order(c.handle, None, 7, None, None, None) == -1   # CS_EINVAL


def test_newton_options_are_checked():
    c = CS.Circuit.from_netlist(G.workload(0))
    assert CS.lib().cs_set_newton_options(c.handle, 4) == -1   # CS_EINVAL: unknown bit
    assert CS.lib().cs_set_newton_options(None, 0) == -1
    c.set_newton_options(programmed_rows=False, upper_runs=False)
    c.set_newton_options()


@pytest.mark.parametrize("idx", [1, 2])
def test_setup_equals_oracle_full_size(orc, idx):
    circ = G.workload(idx)
    c = CS.Circuit.from_netlist(circ)
    col, C, E = c.colour(circ.exclude)
    ocol, oC, oE = orc.colour(circ, True)
    assert np.array_equal(col, ocol) and (C, E) == (oC, oE)
    c.build_map()
    rp, ci = c.pattern()
    orp, oci = orc.pattern(circ)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    for a, b in zip(c.stamp_map(), orc.stamp_map(circ, orp, oci, ocol, True)):
        assert np.array_equal(a, b)


def test_strict_rule_large_chain_is_greedy():
    # the vdd clique of the paper's rule: C = N + 1 for the chain (N >= 4)
    circ = G.inverter_chain_fast(20_000)
    c = CS.Circuit.from_netlist(circ)
    col, C, _ = c.colour(None)
    assert C == 20_001
    assert len(set(col[circ.pol < 0].tolist())) == 20_000


def test_error_paths():
    L = CS.lib()
    circ = G.workload(0)
    bad = circ.term.copy()
    bad[3, 1] = circ.n_nodes
    with pytest.raises(CS.CsError) as e:
        CS.Circuit(circ.n_nodes, bad, circ.pol, circ.vsrc, circ.vsrc_volts)
    assert e.value.status == -1
    badp = circ.pol.copy()
    badp[0] = 0
    with pytest.raises(CS.CsError) as e:
        CS.Circuit(circ.n_nodes, circ.term, badp, circ.vsrc, circ.vsrc_volts)
    assert e.value.status == -1
    c = CS.Circuit.from_netlist(circ)
    with pytest.raises(CS.CsError) as e:
        c.build_map()                       # before colouring
    assert e.value.status == -4
    c.colour(circ.exclude)
    with pytest.raises(CS.CsError) as e:
        c.pattern()                         # before the map
    assert e.value.status == -4
    c.build_map()
    with pytest.raises(CS.CsError) as e:
        c.set_launch(100, 0)
    assert e.value.status == -1
    # evaluate before models/params: state error, no launch
    import ctypes
    st = L.cs_eval_stamp(c.handle, 0, ctypes.c_void_p(1), 0.0, None, ctypes.c_void_p(1),
                         ctypes.c_void_p(1), None)
    assert st == -4
    # the no-allocation form checks the same state first
    assert L.cs_eval_stamp_noalloc(c.handle, ctypes.c_void_p(1), 0.0, None, ctypes.c_void_p(1),
                                   ctypes.c_void_p(1), None) == -4
    assert L.cs_eval_stamp_noalloc(None, ctypes.c_void_p(1), 0.0, None, ctypes.c_void_p(1),
                                   ctypes.c_void_p(1), None) == -1
    assert L.cs_circuit_create(3, 1, None, None, 0, None, None, ctypes.byref(ctypes.c_void_p())) == -1
    bad_card = CS.make_card(G.default_card(1))
    bad_card.size = 3
    assert L.cs_set_models(c.handle, ctypes.byref(bad_card), ctypes.byref(bad_card)) == -1


def test_largest_first_reaches_the_sram_wordline_clique():
    # each wordline gates 512 access transistors: 512 colours are needed, and the
    # largest-first order attains them (the ascending order needs 516)
    circ = G.workload(2)
    c = CS.Circuit.from_netlist(circ)
    assert c.colour(circ.exclude, "largest_first")[1] == 512


def test_random_netlist_covers_every_terminal_pattern():
    # the 52 ways four terminals can coincide or sit on ground (stamp patterns)
    def key(t):
        t0, t1, t2, t3 = (int(v) for v in t)
        c0 = 1 if t0 == 0 else 0
        c1 = 2 if t1 == 0 else (0 if t1 == t0 else 1)
        c2 = 3 if t2 == 0 else (0 if t2 == t0 else (1 if t2 == t1 else 2))
        c3 = 4 if t3 == 0 else (0 if t3 == t0 else (1 if t3 == t1 else (2 if t3 == t2 else 3)))
        return c0 + 2 * (c1 + 3 * (c2 + 4 * c3))
    every = {key(t) for t in itertools.product(range(5), repeat=4)}
    assert len(every) == 52
    assert {key(t) for t in G.random_netlist(600, 6, 21).term} == every


def test_resistor_errors():
    import ctypes
    L = CS.lib()
    circ = G.split_nets(G.ripple_adder28(1), "all")[0]
    c = CS.Circuit.from_netlist(circ)
    bad = circ.res.copy()
    bad[4, 1] = circ.n_nodes
    with pytest.raises(CS.CsError) as e:
        c.set_resistors(bad, circ.res_g)
    assert e.value.status == -1
    g = circ.res_g.copy()
    g[2] = np.nan
    with pytest.raises(CS.CsError) as e:
        c.set_resistors(circ.res, g)
    assert e.value.status == -1
    assert L.cs_set_resistors(c.handle, 3, None, None) == -1
    assert L.cs_set_resistors(c.handle, -1, None, None) == -1
    c.set_resistors(circ.res, circ.res_g)
    c.colour(None)
    c.build_map()
    with pytest.raises(CS.CsError) as e:
        c.set_resistors(circ.res, circ.res_g)     # after the map
    assert e.value.status == -4
    # the pattern grows by the resistors' off-diagonal pairs (every pair is new here)
    p = CS.Circuit.from_netlist(circ)
    p.set_resistors(np.zeros((0, 2), np.int32), np.zeros(0))
    p.colour(None)
    assert c.nnz - p.build_map()[1] == 2 * int(np.count_nonzero(circ.res.min(axis=1)))


def test_junction_cards_are_checked():
    c = CS.Circuit.from_netlist(G.workload(0))
    c.colour(None)
    c.build_map()
    for bad in (dict(pb=0.0), dict(fc=1.0), dict(nj=-1.0), dict(vjmax=2.0), dict(js=-1e-4)):
        with pytest.raises(CS.CsError) as e:
            c.set_models(G.junction_card(1, **bad), G.junction_card(-1))
        assert e.value.status == -1
    c.set_models(G.junction_card(1), G.junction_card(-1))
    c.set_models(G.default_card(1, ), dict(G.default_card(-1), pb=0.0))   # junctions off: not checked


# ---- the binding's tensor checks (they run before any library call) ------------------

def _bad_tensors(n):
    """(tensor, exception) pairs that the binding must refuse for an n-element
    device operand, each before anything reaches the library."""
    import torch
    return [
        (np.zeros(n), TypeError),                                     # not a torch tensor
        (torch.zeros(n, dtype=torch.float32), TypeError),             # wrong dtype
        (torch.zeros(n, dtype=torch.int64), TypeError),
        (torch.zeros(max(n - 1, 0), dtype=torch.float64), ValueError),  # one element short
        (torch.zeros(n + 1, dtype=torch.float64), ValueError),          # one element long
        (torch.zeros(2 * n, dtype=torch.float64)[::2], ValueError),     # not contiguous
        (torch.zeros(n, dtype=torch.float64), ValueError),              # host memory
    ]


def _prepared_chain():
    circ = G.workload(0)
    c = CS.prepare(circ, exclude=True)
    return circ, c


@pytest.mark.parametrize("k", range(7))
def test_binding_refuses_bad_parameter_tensors(k):
    import torch
    circ, c = _prepared_chain()
    n = circ.n_dev
    good = torch.zeros(n, dtype=torch.float64)   # host memory: never reaches the library either
    bad, exc = _bad_tensors(n)[k]
    with pytest.raises(exc):
        c.set_params(bad, good, good)
    with pytest.raises((TypeError, ValueError)):
        c.set_params(good, good, bad)


@pytest.mark.parametrize("k", range(7))
def test_binding_refuses_bad_step_operands(k):
    import torch
    circ, c = _prepared_chain()
    for what, n in (("x", c.n_rows), ("A", c.nnz), ("b", c.n_rows), ("hist", 4 * c.n_dev)):
        bad, exc = _bad_tensors(n)[k]
        x = bad if what == "x" else torch.zeros(c.n_rows, dtype=torch.float64)
        kw = {what: bad} if what != "x" else {}
        if what == "hist":
            kw = dict(hist=bad)
        with pytest.raises(exc):
            if what in ("A", "b"):
                c.eval_stamp(torch.zeros(c.n_rows, dtype=torch.float64), 1e12, None,
                             bad if what == "A" else torch.zeros(c.nnz, dtype=torch.float64),
                             bad if what == "b" else torch.zeros(c.n_rows, dtype=torch.float64))
            elif what == "hist":
                c.eval_stamp(torch.zeros(c.n_rows, dtype=torch.float64), 1e12, bad,
                             torch.zeros(c.nnz, dtype=torch.float64), torch.zeros(c.n_rows, dtype=torch.float64))
            else:
                c.eval_stamp(x, 1e12, None, torch.zeros(c.nnz, dtype=torch.float64),
                             torch.zeros(c.n_rows, dtype=torch.float64))


def test_binding_refuses_bad_cotangents_and_batch_operands():
    import torch
    circ, c = _prepared_chain()
    z = lambda m: torch.zeros(m, dtype=torch.float64)
    with pytest.raises(TypeError):
        c.vjp(z(c.n_rows), 1e12, torch.zeros(c.nnz, dtype=torch.float32), z(c.n_rows))
    with pytest.raises(ValueError):
        c.vjp(z(c.n_rows), 1e12, z(c.nnz - 1), z(c.n_rows))
    with pytest.raises(ValueError):
        c.history(z(c.n_rows + 3), 1e12, z(4 * c.n_dev))
    with pytest.raises(ValueError):
        c.newton(z(c.n_rows), 1e12, None, A=z(c.nnz), b=z(c.n_rows - 1))
    B = CS.Batch([c, CS.prepare(G.workload(0), exclude=True)])
    with pytest.raises(ValueError):
        B.set_params(z(B.n_dev - 1), z(B.n_dev), z(B.n_dev))
    with pytest.raises(TypeError):
        B.set_params(torch.zeros(B.n_dev, dtype=torch.float32), z(B.n_dev), z(B.n_dev))
    with pytest.raises(ValueError):
        B.eval_stamp(z(B.n_rows), 1e12, None, z(B.nnz + 1), z(B.n_rows))
    with pytest.raises(ValueError):
        B.vjp(z(B.n_rows), 1e12, z(B.nnz), z(2 * B.n_rows))
    with pytest.raises(ValueError):
        B.tune(z(B.n_dev), z(B.n_dev), z(B.n_dev), z(B.n_rows), 1e12, z(B.nnz), z(B.n_rows))


def test_handles_close_once_and_exit_hook_closes_the_rest():
    # an explicit close and the exit hook both leave the handle closed, and neither
    # calls the library twice for one handle
    _, c = _prepared_chain()
    B = CS.Batch([c])
    c2 = CS.prepare(G.workload(0), exclude=True)
    B.close()
    B.close()
    c.close()
    assert c.handle is None and B._h is None
    CS._close_all()
    assert c2.handle is None
    c2.close()
