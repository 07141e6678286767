"""GPU parity of the evaluate-and-stamp path (through the C-ABI) against the oracle.

Bars: the coloured variants (persistent, per-colour kernels, buffered, region) reproduce the
oracle's colour replay bit for bit; the atomic variant (no colour order) agrees with
the oracle's serial order within 1e-12 of the per-entry sum of |contributions|
(the reordering bound).  Cases span several workgroups and ragged tails, both
conflict rules, history terms, the empty circuit and the full workload sizes, and
split netlists whose series resistors add a linear part after the FETs."""
import sys

import numpy as np
import pytest

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


def gpu_stamp(torch, circ, exclude, variant, ag0=1e12, hist=None, block=0, eval_ahead=-1, cooperative=True,
              repeat=1, order="natural"):
    c = CS.prepare(circ, exclude, order=order)
    c.set_launch(block, eval_ahead, cooperative)
    dev = torch.device("cuda:0")
    W = torch.from_numpy(circ.W).to(dev)
    L = torch.from_numpy(circ.L).to(dev)
    V = torch.from_numpy(circ.VTH0).to(dev)
    x = torch.from_numpy(circ.x).to(dev)
    h = None if hist is None else torch.from_numpy(np.ascontiguousarray(hist)).to(dev)
    c.set_params(W, L, V)
    A = torch.full((c.nnz,), float("nan"), dtype=torch.float64, device=dev)
    b = torch.full((c.n_rows,), float("nan"), dtype=torch.float64, device=dev)
    for _ in range(repeat):
        c.eval_stamp(x, ag0, h, A, b, variant=variant)
    torch.cuda.synchronize()
    c.check()
    return A.cpu().numpy(), b.cpu().numpy(), c


def oracle_replay(orc, circ, exclude, ag0=1e12, hist=None):
    rp, ci = orc.pattern(circ)
    col, _, _ = orc.colour(circ, exclude)
    return orc.assemble(circ, rp, ci, NC, PC, ag0, hist, col=col, exclude=exclude)


def bits(a):
    return np.ascontiguousarray(a).view(np.int64)


def assert_bit_exact(got, ref, what):
    g, r = bits(got), bits(ref)
    bad = np.nonzero(g != r)[0]
    assert bad.size == 0, f"{what}: {bad.size} entries differ, first {bad[:5]}: {got[bad[:5]]} vs {ref[bad[:5]]}"


def small_cases():
    rng = np.random.default_rng(77)
    out = [
        ("chain50", G.workload(0)),
        ("chain1", G.chain_case(1, 3)),
        ("chain333", G.chain_case(333, 4)),
        ("ota5t", G.draw_params(G.ota5t(), rng, G.W_OPAMP, G.L_OPAMP)),
        ("ring501", G.draw_params(G.ring_oscillator(501), rng, G.W_CHAIN, G.L_CHAIN)),
        ("sram16x16", G.sram_case(16, 16, 5)),
        ("sram3x40", G.sram_case(3, 40, 6)),
        ("pchain50x6", G.draw_params(G.parallel_chain(50, 6), rng, G.W_CHAIN, G.L_CHAIN)),
        ("pchain40x33", G.draw_params(G.parallel_chain(40, 33), rng, G.W_CHAIN, G.L_CHAIN)),
        ("private700", G.draw_params(G.no_shared_nets(700), rng, G.W_CHAIN, G.L_CHAIN)),
        ("adder64x28", G.draw_params(G.ripple_adder28(64), rng, G.W_CHAIN, G.L_CHAIN)),
        # every coincidence pattern of the four terminals, degenerate devices included
        ("random600x6", G.draw_params(G.random_netlist(600, 6, 21), rng, G.W_CHAIN, G.L_CHAIN)),
        # every net split (one colour; PMOS with four distinct nodes: 20 codes)
        ("adder8r89", G.draw_params(G.split_nets(G.ripple_adder28(8), "all")[0], rng, G.W_CHAIN, G.L_CHAIN)),
        # vdd connections split (the resistors' vdd ends are an entry no FET writes)
        ("adder8r14", G.draw_params(G.split_nets(G.ripple_adder28(8), "rail")[0], rng, G.W_CHAIN, G.L_CHAIN)),
        # resistors on FET-written, rail (hub) and new entries, self-loops and ground
        ("random600x6r", G.with_random_resistors(G.draw_params(G.random_netlist(600, 6, 24), rng, G.W_CHAIN,
                                                                G.L_CHAIN), 300, 25)),
    ]
    for k in range(8, 15):
        out.append((f"opamp{k}", G.draw_params(G.opamp2(k, 0.9), rng, G.W_OPAMP, G.L_OPAMP)))
    # regions with more items (entries shared with other regions) than threads: the
    # region schedule counts their arrivals in several rounds (tests/test_region_plan.py
    # checks that the plans have such regions)
    out.append(("random2000x800", G.draw_params(G.random_netlist(2000, 800, 31), np.random.default_rng(78),
                                                G.W_CHAIN, G.L_CHAIN)))
    return out


SMALL = small_cases()


@pytest.mark.parametrize("name,circ", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("exclude", [True, False])
def test_coloured_variants_bit_exact(torch_dev, orc, name, circ, exclude):
    A0, b0 = oracle_replay(orc, circ, exclude)
    for variant, block, ea in (("persistent", 256, 0), ("persistent", 64, 1), ("persistent", 128, -1),
                               ("per_kernel", 0, -1), ("buffered", 0, -1), ("region", 256, -1),
                               ("region", 64, -1), ("region", 192, -1)):
        say(f"case {name} exclude={exclude} variant={variant} block={block} eval_ahead={ea}")
        A, b, _ = gpu_stamp(torch_dev, circ, exclude, variant, block=block, eval_ahead=ea)
        assert_bit_exact(A, A0, f"{name}/{variant}/A")
        assert_bit_exact(b, b0, f"{name}/{variant}/b")


@pytest.mark.parametrize("name,circ", SMALL, ids=[s[0] for s in SMALL])
def test_atomic_within_reordering_bound(torch_dev, orc, name, circ):
    rp, ci = orc.pattern(circ)
    As, bs = orc.assemble(circ, rp, ci, NC, PC, 1e12)
    mA, mb = orc.assemble_magnitude(circ, rp, ci, NC, PC, 1e12)
    for exclude in (True, False):
        for variant in ("atomic", "atomic_wave"):
            say(f"case {name} exclude={exclude} variant={variant}")
            A, b, _ = gpu_stamp(torch_dev, circ, exclude, variant)
            assert np.all(np.abs(A - As) <= 1e-12 * mA), variant
            assert np.all(np.abs(b - bs) <= 1e-12 * mb), variant


SERIAL = SMALL[:9] + [s for s in SMALL if s[0] in ("adder8r89", "adder8r14", "random600x6r")]


@pytest.mark.parametrize("name,circ", SERIAL, ids=[s[0] for s in SERIAL])
def test_serial_stamp_equals_serial_order(torch_dev, orc, name, circ):
    # buffered evaluation, then one lane adds the devices in ascending index onto
    # zeroed A and b: bitwise the oracle's serial accumulation (hubs included)
    rp, ci = orc.pattern(circ)
    As, bs = orc.assemble(circ, rp, ci, NC, PC, 1e12)
    for exclude in (True, False):
        say(f"case {name} exclude={exclude} variant=serial")
        A, b, _ = gpu_stamp(torch_dev, circ, exclude, "serial")
        assert_bit_exact(A, As, f"{name}/serial/A")
        assert_bit_exact(b, bs, f"{name}/serial/b")


@pytest.mark.parametrize("order", ["largest_first", "dsatur"])
def test_other_colouring_orders_bit_exact(torch_dev, orc, order):
    # any proper colouring fixes a colour order; every coloured variant reproduces the
    # oracle's replay in the order of the oracle's own colouring of that kind
    cases = [("chain50", G.workload(0), False), ("sram16x16", G.sram_case(16, 16, 5), True),
             ("adder64x28", G.adder_case(64, 9), False), ("pchain50x6", SMALL[7][1], True)]
    for name, circ, exclude in cases:
        rp, ci = orc.pattern(circ)
        col, _, _ = orc.colour_order(circ, exclude, order)
        A0, b0 = orc.assemble(circ, rp, ci, NC, PC, 1e12, col=col, exclude=exclude)
        for variant, block in (("region", 256), ("region", 64), ("persistent", 256), ("per_kernel", 0)):
            say(f"case {name} exclude={exclude} order={order} variant={variant} block={block}")
            A, b, _ = gpu_stamp(torch_dev, circ, exclude, variant, block=block, order=order)
            assert_bit_exact(A, A0, f"{name}/{order}/{variant}/A")
            assert_bit_exact(b, b0, f"{name}/{order}/{variant}/b")


def test_history_and_dc(torch_dev, orc):
    circ = G.workload(0)
    rng = np.random.default_rng(3)
    hist = rng.normal(0.0, 1e-5, (circ.n_dev, 4))
    for ag0, h in ((1e12, hist), (0.0, None), (3.7e11, hist)):
        A0, b0 = oracle_replay(orc, circ, True, ag0, h)
        for variant in ("persistent", "per_kernel", "region"):
            say(f"case chain50 ag0={ag0} hist={h is not None} variant={variant}")
            A, b, _ = gpu_stamp(torch_dev, circ, True, variant, ag0=ag0, hist=h)
            assert_bit_exact(A, A0, "A")
            assert_bit_exact(b, b0, "b")


def test_empty_circuit(torch_dev, orc):
    circ = G.Circuit("empty", 3, np.zeros((0, 4), np.int32), np.zeros(0, np.int8),
                     np.array([[1, 0]], np.int32), np.array([1.1]), np.array([0, 1, 0], np.uint8), 1.1,
                     np.zeros(0), np.zeros(0), np.zeros(0), np.array([1.1, 0.3, 0.0]))
    for variant in ("persistent", "per_kernel", "atomic", "buffered", "region", "serial"):
        say(f"case empty variant={variant}")
        A, b, _ = gpu_stamp(torch_dev, circ, True, variant)
        # rows: vdd, node 2, branch; entries: (vdd,vdd), (vdd,br), (2,2), (br,vdd)
        assert A.tolist() == [0.0, 1.0, 0.0, 1.0] and b.tolist() == [0.0, 0.0, 1.1]


def test_repeated_calls_are_deterministic(torch_dev, orc):
    circ = G.sram_case(32, 8, 11)
    for variant in ("persistent", "region"):
        A1, b1, _ = gpu_stamp(torch_dev, circ, True, variant, repeat=1)
        A2, b2, _ = gpu_stamp(torch_dev, circ, True, variant, repeat=3)
        assert_bit_exact(A1, A2, "A")
        assert_bit_exact(b1, b2, "b")


@pytest.mark.parametrize("idx", [1, 2])
def test_full_size_workloads(torch_dev, orc, idx):
    circ = G.workload(idx)
    A0, b0 = oracle_replay(orc, circ, True)
    variants = [("persistent", 256, -1), ("persistent", 256, 0), ("per_kernel", 0, -1),
                ("buffered", 0, -1), ("region", 256, -1), ("region", 128, -1)]
    for variant, block, ea in variants:
        say(f"case workload{idx} variant={variant} eval_ahead={ea}")
        A, b, c = gpu_stamp(torch_dev, circ, True, variant, block=block, eval_ahead=ea)
        say("  info", c.info())
        assert_bit_exact(A, A0, f"workload{idx}/{variant}/A")
        assert_bit_exact(b, b0, f"workload{idx}/{variant}/b")
    rp, ci = orc.pattern(circ)
    As, bs = orc.assemble(circ, rp, ci, NC, PC, 1e12)
    mA, mb = orc.assemble_magnitude(circ, rp, ci, NC, PC, 1e12)
    for variant in ("atomic", "atomic_wave"):
        say(f"case workload{idx} variant={variant}")
        A, b, _ = gpu_stamp(torch_dev, circ, True, variant)
        assert np.all(np.abs(A - As) <= 1e-12 * mA), variant
        assert np.all(np.abs(b - bs) <= 1e-12 * mb), variant


def test_full_size_strict_chain(torch_dev, orc):
    # rails not excluded: 100,001 colours; the vdd diagonal and vdd RHS row take one
    # contribution per PMOS, folded in colour order by the follow-up kernel (in the
    # grid-barrier form too, where they take no level)
    circ = G.workload(1)
    A0, b0 = oracle_replay(orc, circ, False)
    for variant, block, ea in (("region", 256, -1), ("region", 128, -1), ("persistent", 256, 1)):
        say(f"case workload1 strict variant={variant} block={block} eval_ahead={ea}")
        A, b, c = gpu_stamp(torch_dev, circ, False, variant, block=block, eval_ahead=ea)
        assert_bit_exact(A, A0, f"strict/{variant}{block}/A")
        assert_bit_exact(b, b0, f"strict/{variant}{block}/b")


@pytest.mark.parametrize("variant", ["persistent", "per_kernel", "buffered", "atomic", "region"])
def test_graph_replay_matches_eager(torch_dev, orc, variant):
    # The NR step captured once and replayed; x changes between replays (eager work
    # in between); every replay must equal the oracle at that x.
    torch = torch_dev
    circ = G.sram_case(12, 20, 21)
    c = CS.prepare(circ, True)
    dev = torch.device("cuda:0")
    c.set_params(*(torch.from_numpy(a).to(dev) for a in (circ.W, circ.L, circ.VTH0)))
    x = torch.from_numpy(circ.x).to(dev)
    A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
    b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)
    c.eval_stamp(x, 1e12, None, A, b, variant)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c.eval_stamp(x, 1e12, None, A, b, variant)
    rng = np.random.default_rng(5)
    for rep in range(3):
        xs = circ.x.copy()
        xs[1:circ.n_nodes - 1] = rng.uniform(0.0, circ.vdd, circ.n_nodes - 2)
        x.copy_(torch.from_numpy(xs))
        A.fill_(float("nan"))
        say(f"case graph replay {rep} variant={variant}")
        g.replay()
        torch.cuda.synchronize()
        c.check()
        rp, ci = orc.pattern(circ)
        if variant == "atomic":
            As, bs = orc.assemble(circ, rp, ci, NC, PC, 1e12, x=xs)
            assert np.allclose(A.cpu().numpy(), As, rtol=1e-12, atol=1e-18)
            continue
        col, _, _ = orc.colour(circ, True)
        A0, b0 = orc.assemble(circ, rp, ci, NC, PC, 1e12, col=col, exclude=True, x=xs)
        assert_bit_exact(A.cpu().numpy(), A0, f"replay{rep}/A")
        assert_bit_exact(b.cpu().numpy(), b0, f"replay{rep}/b")


def test_ordinary_launch_bit_exact(torch_dev, orc):
    for idx in (0, 1):
        circ = G.workload(idx)
        A0, b0 = oracle_replay(orc, circ, True)
        for ea in (0, 1):
            say(f"case workload{idx} ordinary launch eval_ahead={ea}")
            A, b, _ = gpu_stamp(torch_dev, circ, True, "persistent", eval_ahead=ea, cooperative=False)
            assert_bit_exact(A, A0, "A")
            assert_bit_exact(b, b0, "b")
