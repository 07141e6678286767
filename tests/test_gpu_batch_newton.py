"""Batched Newton loop (cs_batch_newton): one Newton step of every circuit of a batch
per iteration, the packed block-diagonal system stamped by cs_batch_eval_stamp and
solved at once, against the oracle's Newton loop run on each circuit alone.

The batch stops when its largest step is <= tol, so a circuit that converged early
keeps taking steps below rounding; every circuit's converged point agrees with the
oracle's within 1e-9 and the batch's iteration count is the largest of the oracle's
within one.  A batch of one circuit orders, factors and solves exactly as cs_newton
does on that circuit: the iterates are the same bits."""
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


def members():
    adder = G.draw_params(G.split_nets(G.drive(G.drive(G.drive(G.ripple_adder28(4), 2, 1.0), 3, 0.0), 4, 1.0),
                                       "all")[0], np.random.default_rng(8), G.W_CHAIN, G.L_CHAIN)
    return [G.chain_dc_case(300, 21, 0.3), adder, G.chain_dc_case(2000, 7, 0.3), G.chain_dc_case(40, 6, 1.0),
            G.draw_params(G.split_nets(G.ripple_adder28(4), "rail")[0], np.random.default_rng(9), G.W_CHAIN,
                          G.L_CHAIN)]


def batch_of(torch, circs):
    B = CS.Batch([CS.prepare(c, True, NC, PC) for c in circs])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    B.set_params(t(np.concatenate([c.W for c in circs])), t(np.concatenate([c.L for c in circs])),
                 t(np.concatenate([c.VTH0 for c in circs])))
    return B, t


@pytest.mark.parametrize("solver,schedule", [("levels", "persistent"), ("rocsolver", "persistent"),
                                             ("levels", "region")])
def test_batch_newton_matches_oracle_per_circuit(torch_dev, solver, schedule):
    circs = members()
    hists = [np.random.default_rng(40 + i).normal(0, 1e-5, (c.n_dev, 4)) for i, c in enumerate(circs)]
    ref = [ON.newton(c, NC, PC, ag0=1e12, hist=h) for c, h in zip(circs, hists)]
    assert all(r[2][-1] <= 1e-9 for r in ref), "oracle did not converge"
    B, t = batch_of(torch_dev, circs)
    B.set_launch(block=256, schedule=schedule)
    x = t(np.concatenate([c.x for c in circs])).clone()
    say(f"case batch newton {len(circs)} circuits, {B.n_rows} rows, solver={solver}, stamp schedule={schedule}")
    r = B.newton(x, 1e12, t(np.concatenate(hists)), solver=solver)
    torch_dev.cuda.synchronize()
    say("  ", r)
    assert r["converged"] and abs(r["iterations"] - max(it for _, it, _ in ref)) <= 1
    xs = x.cpu().numpy()
    for i, (xo, _, _) in enumerate(ref):
        got = xs[B.row_off[i]:B.row_off[i + 1]]
        assert np.abs(got - xo).max() <= 1e-9, f"circuit {i}"


def test_batch_of_one_is_cs_newton_bit_for_bit(torch_dev):
    circ = G.chain_dc_case(2000, 7, 0.3)
    hist = np.random.default_rng(11).normal(0, 1e-5, (circ.n_dev, 4))
    B, t = batch_of(torch_dev, [circ])
    xb = t(circ.x).clone()
    say("case batch newton of one chain2000")
    rb = B.newton(xb, 1e12, t(hist))
    c = CS.prepare(circ, True, NC, PC)
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    xc = t(circ.x).clone()
    rc = c.newton(xc, 1e12, t(hist))
    torch_dev.cuda.synchronize()
    assert rb["iterations"] == rc["iterations"] and rb["converged"]
    assert np.array_equal(xb.cpu().numpy().view(np.int64), xc.cpu().numpy().view(np.int64))


def test_batch_newton_reuses_its_factor_and_reports_non_convergence(torch_dev):
    circs = members()[:3]
    B, t = batch_of(torch_dev, circs)
    x0 = t(np.concatenate([c.x for c in circs]))
    x = x0.clone()
    say("case batch newton max_iter=1, then a full solve on the same state")
    r = B.newton(x, 1e12, None, max_iter=1)
    assert r["iterations"] == 1 and not r["converged"] and r["last_step"] > 1e-9
    assert r["ms"]["host_factor"] > 0.0
    x = x0.clone()
    r2 = B.newton(x, 1e12, None)
    torch_dev.cuda.synchronize()
    assert r2["converged"]
    for i, c in enumerate(circs):
        xo, _, steps = ON.newton(c, NC, PC, ag0=1e12)
        assert steps[-1] <= 1e-9
        assert np.abs(x.cpu().numpy()[B.row_off[i]:B.row_off[i + 1]] - xo).max() <= 1e-9


def test_batch_history_is_per_circuit_history(torch_dev):
    circs = members()[:2]
    B, t = batch_of(torch_dev, circs)
    B.per_circuit_params(t(np.concatenate([c.W for c in circs])), t(np.concatenate([c.L for c in circs])),
                         t(np.concatenate([c.VTH0 for c in circs])))
    x = t(np.concatenate([c.x for c in circs]))
    say("case batch history")
    got = B.history(x, 1e12).cpu().numpy()
    ref = np.concatenate([ON.history(c, NC, PC, c.x, 1e12) for c in circs])
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


@pytest.mark.parametrize("solver", ["levels", "rocsolver"])
def test_batch_transient_matches_oracle_per_circuit(torch_dev, solver):
    # three 20-stage chains (inputs held high, low, high; different random starts and
    # sizes) stepped together for 40 steps of 1 ps: each waveform within 1e-7 V of the
    # oracle's transient of that chain alone
    circs = [G.chain_dc_case(20, seed=15, vin=1.0), G.chain_dc_case(20, seed=16, vin=0.0),
             G.chain_dc_case(12, seed=17, vin=1.0)]
    refs = [ON.transient(c, NC, PC, 1e-12, 40)[0] for c in circs]
    B, t = batch_of(torch_dev, circs)
    B.per_circuit_params(t(np.concatenate([c.W for c in circs])), t(np.concatenate([c.L for c in circs])),
                         t(np.concatenate([c.VTH0 for c in circs])))
    x = t(np.concatenate([c.x for c in circs])).clone()
    say(f"case batch transient 3 chains solver={solver}")
    wave, iters = B.transient(x, 1e-12, 40, solver=solver)
    wave = wave.cpu().numpy()
    for i, ref in enumerate(refs):
        got = wave[:, B.row_off[i]:B.row_off[i + 1]]
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() <= 1e-7, f"circuit {i}"
