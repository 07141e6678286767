"""GPU checks of the batched kernel and of the adjoint.

Batch: one launch over many circuits reproduces every circuit's oracle colour
replay bit for bit, for every launch configuration the autotuner can pick, and
equals the per-circuit launches.  Adjoint: the hand-written VJP of (A, b) with
respect to W, L, VTH0 agrees with the oracle's complex-step gradient within 1e-8 of
the per-device scale sum |cotangent * sensitivity| (plus 8 ulps of the device's
rounding scale, where the oracle's own value is decided by rounding: vjpbound), and
with central differences (step 1e-6 relative) of the GPU forward within 1e-6."""
import sys

import numpy as np
import pytest
import vjpbound

from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

pytestmark = pytest.mark.gpu
NC, PC = G.default_card(1), G.default_card(-1)


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    CS.lib()
    return torch


def bits(a):
    return np.ascontiguousarray(a).view(np.int64)


def small_batch():
    return G.batch_sweep(seed=9, n_opamp=40, n_chain=8, n_ring=5, chain_range=(50, 1500),
                         ring_range=(301, 2501))


def packed(torch, circs, attr):
    return torch.from_numpy(np.concatenate([getattr(c, attr) for c in circs])).to("cuda:0")


@pytest.fixture(scope="module")
def batch_oracle(orc):
    circs = small_batch()
    ref = []
    for c in circs:
        rp, ci = orc.pattern(c)
        col, _, _ = orc.colour(c, True)
        ref.append(orc.assemble(c, rp, ci, NC, PC, 1e12, col=col, exclude=True))
    return circs, ref


@pytest.mark.parametrize("block,eval_ahead,local,schedule", [
    (256, -1, 0, "persistent"), (128, 0, 0, "persistent"), (256, 0, 64, "persistent"),
    (256, -1, 256, "persistent"), (64, 0, 10 ** 9, "persistent"), (256, 1, 400, "persistent"),
    (256, -1, 0, "region"), (128, -1, 0, "region"), (64, -1, 0, "region")])
def test_batch_bit_exact_per_circuit(torch_dev, batch_oracle, block, eval_ahead, local, schedule):
    torch = torch_dev
    circs, ref = batch_oracle
    cs = [CS.prepare(c, True) for c in circs]
    B = CS.Batch(cs)
    B.set_launch(block, eval_ahead, local, schedule)
    W, L, V, x = (packed(torch, circs, a) for a in ("W", "L", "VTH0", "x"))
    B.set_params(W, L, V)
    A = torch.full((B.nnz,), float("nan"), dtype=torch.float64, device="cuda:0")
    b = torch.full((B.n_rows,), float("nan"), dtype=torch.float64, device="cuda:0")
    say(f"case batch {schedule} block={block} eval_ahead={eval_ahead} local={local} n_dev={B.n_dev}")
    for _ in range(2):
        B.eval_stamp(x, 1e12, None, A, b)
    torch.cuda.synchronize()
    B.check()
    say("  info", B.info())
    Ah, bh = A.cpu().numpy(), b.cpu().numpy()
    for i, (A0, b0) in enumerate(ref):
        z0, z1 = B.nnz_off[i], B.nnz_off[i + 1]
        r0, r1 = B.row_off[i], B.row_off[i + 1]
        assert np.array_equal(bits(Ah[z0:z1]), bits(A0)), f"circuit {i} ({circs[i].name}) A"
        assert np.array_equal(bits(bh[r0:r1]), bits(b0)), f"circuit {i} ({circs[i].name}) b"
    # the per-circuit comparison schedule gives the same bits
    B.per_circuit_params(W, L, V)
    A2 = torch.full_like(A, float("nan"))
    b2 = torch.full_like(b, float("nan"))
    B.per_circuit_eval(x, 1e12, A2, b2)
    torch.cuda.synchronize()
    assert np.array_equal(bits(A2.cpu().numpy()), bits(Ah))
    assert np.array_equal(bits(b2.cpu().numpy()), bits(bh))


def test_autotuner_picks_a_valid_configuration(torch_dev, batch_oracle, tmp_path):
    from paper_2604_03079_amd import autotune
    torch = torch_dev
    circs, ref = batch_oracle
    B = CS.Batch([CS.prepare(c, True) for c in circs])
    W, L, V, x = (packed(torch, circs, a) for a in ("W", "L", "VTH0", "x"))
    A = torch.empty(B.nnz, dtype=torch.float64, device="cuda:0")
    b = torch.empty(B.n_rows, dtype=torch.float64, device="cuda:0")
    say("case autotune")
    best = autotune.tune(B, W, L, V, x, 1e12, A, b, cache_path=str(tmp_path / "t.json"), reps=3)
    assert best["ms"] > 0 and not best["cached"]
    again = autotune.tune(B, W, L, V, x, 1e12, A, b, cache_path=str(tmp_path / "t.json"), reps=3)
    assert again["cached"]
    B.eval_stamp(x, 1e12, None, A, b)
    torch.cuda.synchronize()
    Ah = A.cpu().numpy()
    for i, (A0, _) in enumerate(ref):
        assert np.array_equal(bits(Ah[B.nnz_off[i]:B.nnz_off[i + 1]]), bits(A0))


@pytest.mark.parametrize("schedule", ["persistent", "region"])
def test_batch_with_series_resistors(torch_dev, orc, schedule):
    # split netlists and random resistors in one batch: each circuit's linear part
    # is added after the batched schedule, bitwise the oracle's replay
    torch = torch_dev
    rng = np.random.default_rng(12)
    circs = [G.draw_params(G.split_nets(G.ripple_adder28(3), "all")[0], rng, G.W_CHAIN, G.L_CHAIN),
             G.workload(0),
             G.draw_params(G.split_nets(G.ripple_adder28(2), "rail")[0], rng, G.W_CHAIN, G.L_CHAIN),
             G.with_random_resistors(G.draw_params(G.random_netlist(200, 6, 26), rng, G.W_CHAIN, G.L_CHAIN),
                                     80, 27)]
    ref = []
    for c in circs:
        rp, ci = orc.pattern(c)
        col, _, _ = orc.colour(c, True)
        ref.append(orc.assemble(c, rp, ci, NC, PC, 1e12, col=col, exclude=True))
    B = CS.Batch([CS.prepare(c, True) for c in circs])
    B.set_launch(256, -1, 0, schedule)
    W, L, V, x = (packed(torch, circs, a) for a in ("W", "L", "VTH0", "x"))
    B.set_params(W, L, V)
    A = torch.full((B.nnz,), float("nan"), dtype=torch.float64, device="cuda:0")
    b = torch.full((B.n_rows,), float("nan"), dtype=torch.float64, device="cuda:0")
    say(f"case batch with resistors {schedule} n_dev={B.n_dev}")
    for _ in range(2):
        B.eval_stamp(x, 1e12, None, A, b)
    torch.cuda.synchronize()
    B.check()
    Ah, bh = A.cpu().numpy(), b.cpu().numpy()
    for i, (A0, b0) in enumerate(ref):
        z0, z1 = B.nnz_off[i], B.nnz_off[i + 1]
        r0, r1 = B.row_off[i], B.row_off[i + 1]
        assert np.array_equal(bits(Ah[z0:z1]), bits(A0)), f"circuit {i} ({circs[i].name}) A"
        assert np.array_equal(bits(bh[r0:r1]), bits(b0)), f"circuit {i} ({circs[i].name}) b"


def gpu_vjp(torch, circ, Ab, bb, ag0=1e12):
    c = CS.prepare(circ, True)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    g = c.vjp(t(circ.x), ag0, t(Ab), t(bb))
    torch.cuda.synchronize()
    return [v.cpu().numpy() for v in g], c


VJP_CASES = [("chain50", lambda: G.workload(0)),
             ("opamp12", lambda: G.draw_params(G.opamp2(12), np.random.default_rng(2), G.W_OPAMP, G.L_OPAMP)),
             ("sram6x6", lambda: G.sram_case(6, 6, 8)),
             ("ring301", lambda: G.draw_params(G.ring_oscillator(301), np.random.default_rng(4), G.W_CHAIN, G.L_CHAIN)),
             ("random600x6", lambda: G.draw_params(G.random_netlist(600, 6, 21), np.random.default_rng(31),
                                                   G.W_CHAIN, G.L_CHAIN)),
             # series resistors are constants: the gradients are the FETs' alone
             ("adder4r89", lambda: G.draw_params(G.split_nets(G.ripple_adder28(4), "all")[0],
                                                 np.random.default_rng(32), G.W_CHAIN, G.L_CHAIN))]


@pytest.mark.parametrize("name,make", VJP_CASES, ids=[v[0] for v in VJP_CASES])
def test_vjp_matches_oracle_complex_step(torch_dev, orc, name, make):
    circ = make()
    rp, ci = orc.pattern(circ)
    Ab, bb = G.cotangents(len(ci), circ.n_rows, seed=50)
    ref = orc.vjp(circ, rp, ci, NC, PC, 1e12, Ab, bb)
    say(f"case vjp {name}")
    got, _ = gpu_vjp(torch_dev, circ, Ab, bb)
    worst = vjpbound.check(orc, got, circ, rp, ci, NC, PC, 1e12, Ab, bb, ref=ref, label=name)
    say(f"  worst |d|/sensitivity scale: W {worst[0]:.2e} L {worst[1]:.2e} VTH0 {worst[2]:.2e}")


def test_vjp_full_size_chain10k(torch_dev, orc):
    circ = G.workload(4)
    rp, ci = orc.pattern(circ)
    Ab, bb = G.cotangents(len(ci), circ.n_rows, seed=50)
    say("case vjp chain10000")
    got, _ = gpu_vjp(torch_dev, circ, Ab, bb)
    vjpbound.check(orc, got, circ, rp, ci, NC, PC, 1e12, Ab, bb, label="chain10000")


def test_vjp_matches_central_differences_of_gpu_forward(torch_dev, orc):
    torch = torch_dev
    circ = G.workload(0)
    rp, ci = orc.pattern(circ)
    Ab, bb = G.cotangents(len(ci), circ.n_rows, seed=50)
    (gW, gL, gV), c = gpu_vjp(torch, circ, Ab, bb)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    x = t(circ.x)

    def J(W, L, V):
        c.set_params(t(W), t(L), t(V))
        A, b = c.eval_stamp(x, 1e12, variant="persistent")
        torch.cuda.synchronize()
        return float(Ab @ A.cpu().numpy() + bb @ b.cpu().numpy())

    rng = np.random.default_rng(12)
    base = dict(W=circ.W, L=circ.L, V=circ.VTH0)
    for name, g in (("W", gW), ("L", gL), ("V", gV)):
        d = rng.standard_normal(circ.n_dev)
        h = 1e-6 * np.abs(base[name])
        p = {k: v.copy() for k, v in base.items()}
        m = {k: v.copy() for k, v in base.items()}
        p[name] = p[name] + h * d
        m[name] = m[name] - h * d
        fd = (J(p["W"], p["L"], p["V"]) - J(m["W"], m["L"], m["V"])) / 2.0
        an = float(np.sum(g * h * d))
        scale = float(np.sum(np.abs(g * h * d)))
        say(f"case fd {name}: fd={fd:.6e} adjoint={an:.6e}")
        assert abs(fd - an) <= 1e-6 * scale


def test_autograd_function(torch_dev, orc):
    torch = torch_dev
    circ = G.workload(0)
    c = CS.prepare(circ, True)
    dev = torch.device("cuda:0")
    W = torch.from_numpy(circ.W).to(dev).requires_grad_(True)
    L = torch.from_numpy(circ.L).to(dev).requires_grad_(True)
    V = torch.from_numpy(circ.VTH0).to(dev).requires_grad_(True)
    x = torch.from_numpy(circ.x).to(dev)
    rp, ci = orc.pattern(circ)
    Ab, bb = G.cotangents(len(ci), circ.n_rows, seed=50)
    A, b = CS.stamp(c, W, L, V, x, 1e12)
    loss = (A * torch.from_numpy(Ab).to(dev)).sum() + (b * torch.from_numpy(bb).to(dev)).sum()
    loss.backward()
    vjpbound.check(orc, [g.cpu().numpy() for g in (W.grad, L.grad, V.grad)], circ, rp, ci, NC, PC, 1e12,
                   Ab, bb, label="autograd")


def test_batch_vjp_equals_per_circuit(torch_dev, batch_oracle, orc):
    torch = torch_dev
    circs, _ = batch_oracle
    circs = circs[:12]
    B = CS.Batch([CS.prepare(c, True) for c in circs])
    W, L, V, x = (packed(torch, circs, a) for a in ("W", "L", "VTH0", "x"))
    B.set_params(W, L, V)
    Ab, bb = G.cotangents(B.nnz, B.n_rows, seed=50)
    say("case batch vjp")
    gW, gL, gV = B.vjp(x, 1e12, torch.from_numpy(Ab).to("cuda:0"), torch.from_numpy(bb).to("cuda:0"))
    torch.cuda.synchronize()
    for i, c in enumerate(circs):
        d0, d1 = B.dev_off[i], B.dev_off[i + 1]
        rp, ci = orc.pattern(c)
        Abi = Ab[B.nnz_off[i]:B.nnz_off[i + 1]]
        bbi = bb[B.row_off[i]:B.row_off[i + 1]]
        vjpbound.check(orc, [g.cpu().numpy()[d0:d1] for g in (gW, gL, gV)], c, rp, ci, NC, PC, 1e12, Abi, bbi,
                       label=f"batch circuit {i}")


def test_two_lane_adjoint_equals_one_lane(torch_dev):
    # Below one 256-thread block per compute unit of devices the adjoint gives each
    # device two lanes with one tangent each; above, one lane carries both.  Chains of
    # 1,000 stages alone take the two-lane form, their batch the one-lane form: the
    # same arithmetic per tangent gives the same bits.
    torch = torch_dev
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n_chain = (cus * 256) // 2000 + 2
    circs = [G.chain_case(1000, seed=200 + i) for i in range(n_chain)]
    assert circs[0].n_dev < cus * 256 <= sum(c.n_dev for c in circs)
    B = CS.Batch([CS.prepare(c, True) for c in circs])
    W, L, V, x = (packed(torch, circs, a) for a in ("W", "L", "VTH0", "x"))
    B.set_params(W, L, V)
    Ab, bb = G.cotangents(B.nnz, B.n_rows, seed=51)
    say(f"case two-lane vs one-lane adjoint: {n_chain} chains, {B.n_dev} devices")
    gB = [g.cpu().numpy() for g in B.vjp(x, 1e12, torch.from_numpy(Ab).to("cuda:0"),
                                         torch.from_numpy(bb).to("cuda:0"))]
    for i, c in enumerate(circs):
        d0, d1 = B.dev_off[i], B.dev_off[i + 1]
        g, h = gpu_vjp(torch, c, Ab[B.nnz_off[i]:B.nnz_off[i + 1]], bb[B.row_off[i]:B.row_off[i + 1]])
        h.close()
        for k, name in enumerate(("W", "L", "VTH0")):
            assert np.array_equal(bits(g[k]), bits(gB[k][d0:d1])), f"chain {i} d/d{name}"
    B.close()
