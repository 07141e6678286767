"""GPU Newton loop (cs_newton: stamp, sparse LU refactorisation and solve, damped
update) against the oracle's Newton loop from the same start.

Both sides take the same steps (stamp at x, solve, clamp node rows to +-vstep,
stop at max |step| <= tol); they differ only in how the linear solve rounds, which
the contraction of Newton's method removes: the converged points agree within
1e-9 (the convergence tolerance) and the iteration counts within one.  Cases: DC
operating points of short chains (the symmetric chain at half supply, exact),
backward-Euler steps with history terms on chains and on a split adder with its
series resistors, and the 100,000-stage chain, checked by the KCL residual of the
oracle's stamp at the GPU's point.  Both solvers: the library's level-scheduled
kernels and rocSOLVER's refactorisation with the same pivots.  The history terms of
the next backward-Euler step (ag0 * Q) are bit-exact, and a 60-step transient
follows the oracle's waveform within 1e-7 V."""
import sys

import numpy as np
import pytest

from oracle import newton as ON
from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

pytestmark = pytest.mark.gpu
NC, PC = G.default_card(1), G.default_card(-1)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    CS.lib()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def gpu_newton(torch, circ, ag0=0.0, hist=None, pmos=None, variant="region", **kw):
    c = CS.prepare(circ, True, NC, pmos or PC)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    x = t(circ.x).clone()
    r = c.newton(x, ag0, None if hist is None else t(hist), variant=variant, **kw)
    torch.cuda.synchronize()
    return x.cpu().numpy(), r, c


def test_symmetric_chain_at_half_supply(torch_dev):
    circ = G.drive(G.inverter_chain(2), 2, 0.5)
    n = circ.n_dev
    circ.W, circ.L = np.full(n, 1e-6), np.full(n, 60e-9)
    circ.VTH0 = 0.4 * circ.pol.astype(np.float64)
    circ.x = np.zeros(circ.n_rows)
    circ.x[:circ.n_nodes - 1] = np.random.default_rng(3).uniform(0, 1, circ.n_nodes - 1)
    say("case newton symmetric chain2 DC")
    x, r, _ = gpu_newton(torch_dev, circ, pmos=G.default_card(-1, symmetric=True))
    assert r["converged"]
    assert np.all(np.abs(x[2:circ.n_nodes - 1] - 0.5) <= 1e-12)


CASES = [("chain40dc", lambda: G.chain_dc_case(40, 6, 0.0), 0.0, None),
         ("chain9dc_high", lambda: G.chain_dc_case(9, 5, 1.0), 0.0, None),
         ("chain2000be", lambda: G.chain_dc_case(2000, 7, 0.3), 1e12, 11),
         ("adder4r89be", lambda: G.draw_params(G.split_nets(G.drive(G.drive(G.drive(
             G.ripple_adder28(4), 2, 1.0), 3, 0.0), 4, 1.0), "all")[0], np.random.default_rng(8),
             G.W_CHAIN, G.L_CHAIN), 1e12, 12),
         ("adder4r14be", lambda: G.draw_params(G.split_nets(G.ripple_adder28(4), "rail")[0],
                                               np.random.default_rng(9), G.W_CHAIN, G.L_CHAIN), 1e12, 13)]


@pytest.mark.parametrize("solver", ["levels", "rocsolver"])
@pytest.mark.parametrize("name,make,ag0,hseed", CASES, ids=[c[0] for c in CASES])
def test_newton_matches_oracle(torch_dev, name, make, ag0, hseed, solver):
    circ = make()
    hist = None if hseed is None else np.random.default_rng(hseed).normal(0, 1e-5, (circ.n_dev, 4))
    xo, ito, steps = ON.newton(circ, NC, PC, ag0=ag0, hist=hist)
    assert steps[-1] <= 1e-9, "oracle did not converge"
    say(f"case newton {name} ag0={ag0} solver={solver}")
    x, r, _ = gpu_newton(torch_dev, circ, ag0, hist, solver=solver)
    say("  ", r)
    assert r["converged"] and abs(r["iterations"] - ito) <= 1
    assert np.abs(x - xo).max() <= 1e-9


def test_variants_give_the_same_iterates(torch_dev):
    # the coloured variants stamp bit-identical systems: the loop ends at the same bits
    circ = G.chain_dc_case(2000, 7, 0.3)
    hist = np.random.default_rng(11).normal(0, 1e-5, (circ.n_dev, 4))
    out = []
    for v in ("region", "persistent", "per_kernel", "buffered"):
        say(f"case newton variant {v}")
        x, r, _ = gpu_newton(torch_dev, circ, 1e12, hist, variant=v)
        out.append((x, r["iterations"]))
    for x, it in out[1:]:
        assert it == out[0][1] and np.array_equal(x.view(np.int64), out[0][0].view(np.int64))


@pytest.mark.parametrize("solver", ["levels", "rocsolver"])
def test_full_size_chain_backward_euler_step(torch_dev, orc, solver):
    circ = G.chain_dc_case(100_000, 2, 0.3)
    hist = np.random.default_rng(14).normal(0, 1e-5, (circ.n_dev, 4))
    say(f"case newton chain100k backward Euler solver={solver}")
    x, r, _ = gpu_newton(torch_dev, circ, 1e12, hist, solver=solver)
    say("  ", r)
    assert r["converged"] and r["iterations"] <= 30
    # at the GPU's point the oracle's system satisfies A x = b up to the step size:
    # b = A x - F(x), so the node rows of A x - b are the KCL residual F
    rp, ci = orc.pattern(circ)
    A, b = orc.assemble(circ, rp, ci, NC, PC, 1e12, hist, x=x)
    import scipy.sparse as sp
    M = sp.csr_matrix((A, ci, rp), shape=(circ.n_rows, circ.n_rows))
    F = (M @ x - b)[:circ.n_nodes - 1]
    assert np.abs(F).max() <= 1e-9 * np.abs(M).max()


def test_reports_non_convergence(torch_dev):
    circ = G.chain_dc_case(2000, 7, 0.3)
    say("case newton max_iter=1")
    x, r, _ = gpu_newton(torch_dev, circ, 1e12, None, max_iter=1)
    assert r["iterations"] == 1 and not r["converged"] and r["last_step"] > 1e-9


def test_unknown_solver_is_refused(torch_dev):
    circ = G.chain_dc_case(5, 7, 0.3)
    c = CS.prepare(circ, True)
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    x = t(circ.x)
    A = torch.empty(c.nnz, dtype=torch.float64, device="cuda:0")
    b = torch.empty(c.n_rows, dtype=torch.float64, device="cuda:0")
    assert CS.lib().cs_newton(c.handle, 4, 7, CS._dev_ptr(x), 0.0, None, 10, 0.3, 1e-9, CS._dev_ptr(A),
                              CS._dev_ptr(b), None, None, None, None, None) == -1


@pytest.mark.parametrize("name,make", [("chain50", lambda: G.workload(0)),
                                       ("random600x6", lambda: G.draw_params(G.random_netlist(600, 6, 21),
                                                                             np.random.default_rng(8), G.W_CHAIN,
                                                                             G.L_CHAIN))], ids=["chain50", "random600x6"])
def test_history_terms_bit_exact(torch_dev, name, make):
    # ag0 * Q of every terminal: model M's charges, bit for bit the oracle's
    circ = make()
    c = CS.prepare(circ, True)
    t = lambda a: torch_dev.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    say(f"case history {name}")
    got = c.history(t(circ.x), 1e12).cpu().numpy()
    ref = ON.history(circ, NC, PC, circ.x, 1e12)
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


@pytest.mark.parametrize("solver", ["levels", "rocsolver"])
def test_transient_matches_oracle(torch_dev, solver):
    # 60 backward-Euler steps of 1 ps of a 20-stage chain whose input is held at Vdd,
    # from the generator's random start: the waveforms agree within 1e-7 V
    circ = G.chain_dc_case(20, seed=15, vin=1.0)
    ref, iters_o = ON.transient(circ, NC, PC, 1e-12, 60)
    c = CS.prepare(circ, True)
    t = lambda a: torch_dev.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    x = t(circ.x).clone()
    say(f"case transient chain20 solver={solver}")
    wave, iters = c.transient(x, 1e-12, 60, solver=solver)
    wave = wave.cpu().numpy()
    assert wave.shape == ref.shape
    assert np.abs(wave - ref).max() <= 1e-7
    assert all(abs(a - b) <= 1 for a, b in zip(iters, iters_o))


@pytest.mark.parametrize("name,make", [("adder8r89be", lambda: G.adder_case(8, 9, "all")),
                                       ("chain2000be", lambda: G.chain_dc_case(2000, 7, 0.3))],
                         ids=["adder8r89be", "chain2000be"])
def test_solver_schedules_give_the_same_bits(torch_dev, name, make):
    # programmed rows, runs of narrow lower levels and upper-level runs change the
    # launches, not the arithmetic: each option set gives the same iterates bit for bit
    circ = make()
    hist = np.random.default_rng(16).normal(0, 1e-5, (circ.n_dev, 4))
    t = lambda a: torch_dev.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    c = CS.prepare(circ, True, NC, PC)
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    out = []
    for prog, runs in ((True, True), (False, True), (True, False), (False, False)):
        c.set_newton_options(programmed_rows=prog, upper_runs=runs)
        x = t(circ.x).clone()
        say(f"case newton schedule {name} programmed={prog} upper_runs={runs}")
        r = c.newton(x, 1e12, t(hist))
        torch_dev.cuda.synchronize()
        assert r["converged"]
        out.append((x.cpu().numpy(), r["iterations"]))
    for x, it in out[1:]:
        assert it == out[0][1] and np.array_equal(x.view(np.int64), out[0][0].view(np.int64))
