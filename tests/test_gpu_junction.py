"""GPU parity of the second model level (model M with the source/drain-body
junctions, card jmod = 1) through the same kernels and C-ABI: every coloured
variant bit-exact against the oracle's colour replay, serial stamping against the
serial order, the atomic variant within the reordering bound, the history terms
(junction charges included) bit-exact, the adjoint against the oracle's complex
step, and the Newton loop against the oracle's.  Bias points span reverse, forward
and continued (above vjmax and above fc pb) junction regions."""
import sys

import numpy as np
import pytest
import vjpbound

from oracle import newton as ON
from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

pytestmark = pytest.mark.gpu
NJ, PJ = G.junction_card(1), G.junction_card(-1)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    CS.lib()
    return torch


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def wide_bias(circ, seed):
    # node voltages from -0.4 V to 1.4 V so that junctions see reverse bias, forward
    # bias, and forward bias beyond fc pb (0.5 V) and vjmax (0.8 V)
    rng = np.random.default_rng(seed)
    x = circ.x.copy()
    n = circ.n_nodes - 1
    x[1:n] = rng.uniform(-0.4, 1.4, n - 1)
    circ.x = x
    return circ


CASES = [("chain50", lambda: wide_bias(G.workload(0), 1)),
         ("random600x6", lambda: wide_bias(G.draw_params(G.random_netlist(600, 6, 21), np.random.default_rng(8),
                                                          G.W_CHAIN, G.L_CHAIN), 2)),
         ("sram8x8", lambda: wide_bias(G.sram_case(8, 8, 5), 3)),
         ("adder4r89", lambda: wide_bias(G.draw_params(G.split_nets(G.ripple_adder28(4), "all")[0],
                                                        np.random.default_rng(9), G.W_CHAIN, G.L_CHAIN), 4))]


def tensors(torch, circ):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    return t(circ.W), t(circ.L), t(circ.VTH0), t(circ.x)


def bits(a):
    return np.ascontiguousarray(a).view(np.int64)


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_junction_level_stamp_parity(torch_dev, orc, name, make):
    torch = torch_dev
    circ = make()
    rp, ci = orc.pattern(circ)
    W, L, V, x = tensors(torch, circ)
    for exclude in (True, False):
        col, _, _ = orc.colour(circ, exclude)
        A0, b0 = orc.assemble(circ, rp, ci, NJ, PJ, 1e12, col=col, exclude=exclude)
        c = CS.prepare(circ, exclude, NJ, PJ)
        c.set_params(W, L, V)
        for variant in ("region", "persistent", "per_kernel", "buffered"):
            say(f"case junction {name} exclude={exclude} variant={variant}")
            A, b = c.eval_stamp(x, 1e12, variant=variant)
            torch.cuda.synchronize()
            c.check()
            assert np.array_equal(bits(A.cpu().numpy()), bits(A0)), variant
            assert np.array_equal(bits(b.cpu().numpy()), bits(b0)), variant
    As, bs = orc.assemble(circ, rp, ci, NJ, PJ, 1e12)
    mA, mb = orc.assemble_magnitude(circ, rp, ci, NJ, PJ, 1e12)
    c = CS.prepare(circ, True, NJ, PJ)
    c.set_params(W, L, V)
    say(f"case junction {name} serial, atomic")
    A, b = c.eval_stamp(x, 1e12, variant="serial")
    torch.cuda.synchronize()
    assert np.array_equal(bits(A.cpu().numpy()), bits(As)) and np.array_equal(bits(b.cpu().numpy()), bits(bs))
    A, b = c.eval_stamp(x, 1e12, variant="atomic")
    torch.cuda.synchronize()
    assert np.all(np.abs(A.cpu().numpy() - As) <= 1e-12 * mA)
    assert np.all(np.abs(b.cpu().numpy() - bs) <= 1e-12 * mb)


@pytest.mark.parametrize("name,make", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_junction_level_history_bit_exact(torch_dev, name, make):
    circ = make()
    c = CS.prepare(circ, True, NJ, PJ)
    W, L, V, x = tensors(torch_dev, circ)
    c.set_params(W, L, V)
    say(f"case junction history {name}")
    got = c.history(x, 1e12).cpu().numpy()
    ref = ON.history(circ, NJ, PJ, circ.x, 1e12)
    assert np.array_equal(bits(got), bits(ref))


@pytest.mark.parametrize("name,make", CASES[:2], ids=[c[0] for c in CASES[:2]])
def test_junction_level_vjp(torch_dev, orc, name, make):
    # the junction area follows Weff: the W gradient includes the junction terms
    circ = make()
    rp, ci = orc.pattern(circ)
    Ab, bb = G.cotangents(len(ci), circ.n_rows, seed=50)
    c = CS.prepare(circ, True, NJ, PJ)
    W, L, V, x = tensors(torch_dev, circ)
    c.set_params(W, L, V)
    t = lambda a: torch_dev.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    say(f"case junction vjp {name}")
    got = [g.cpu().numpy() for g in c.vjp(x, 1e12, t(Ab), t(bb))]
    worst = vjpbound.check(orc, got, circ, rp, ci, NJ, PJ, 1e12, Ab, bb, label=name)
    say(f"  worst |d|/sensitivity scale: W {worst[0]:.2e} L {worst[1]:.2e} VTH0 {worst[2]:.2e}")


def test_junction_level_newton(torch_dev):
    circ = G.chain_dc_case(300, seed=16, vin=0.3)
    hist = np.random.default_rng(17).normal(0, 1e-5, (circ.n_dev, 4))
    xo, ito, steps = ON.newton(circ, NJ, PJ, ag0=1e12, hist=hist)
    assert steps[-1] <= 1e-9
    c = CS.prepare(circ, True, NJ, PJ)
    W, L, V, x = tensors(torch_dev, circ)
    c.set_params(W, L, V)
    x = x.clone()
    say("case junction newton chain300")
    r = c.newton(x, 1e12, torch_dev.from_numpy(hist).to("cuda:0"))
    assert r["converged"] and abs(r["iterations"] - ito) <= 1
    assert np.abs(x.cpu().numpy() - xo).max() <= 1e-9
