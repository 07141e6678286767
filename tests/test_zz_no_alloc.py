"""cs_eval_stamp_noalloc, the evaluate-and-stamp for callers that cannot allocate
(its scratch memory in the library's per-GPU array), against cs_eval_stamp with the
region schedule (CS_COLOR_REGION), bit for bit:

* two calls in a row, the second with a smaller circuit (the array keeps the first
  call's contents, counters included), then the first circuit again;
* the call captured in a HIP graph and replayed with new voltages between replays;
* a circuit whose scratch exceeds the array is refused with CS_ENOTSUP before any
  launch, and one whose region tables are not on the device with CS_ESTATE."""
import sys

import numpy as np
import pytest

from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

pytestmark = pytest.mark.gpu
AG0 = 1e12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bits(t):
    return np.ascontiguousarray(t.cpu().numpy()).view(np.int64)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    CS.lib()
    return torch


def setup(torch, circ):
    dev = torch.device("cuda:0")
    c = CS.prepare(circ, True)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    return c, t


def reference(torch, c, x, hist=None):
    A = torch.empty(c.nnz, dtype=torch.float64, device=x.device)
    b = torch.empty(c.n_rows, dtype=torch.float64, device=x.device)
    c.eval_stamp(x, AG0, hist, A, b, "region")
    torch.cuda.synchronize()
    return A, b


def noalloc(torch, c, x, hist=None):
    A = torch.full((c.nnz,), float("nan"), dtype=torch.float64, device=x.device)
    b = torch.full((c.n_rows,), float("nan"), dtype=torch.float64, device=x.device)
    c.eval_stamp_noalloc(x, AG0, A, b, hist)
    torch.cuda.synchronize()
    c.check()
    return A, b


def test_noalloc_equals_region_entry_point_big_then_small(torch_dev):
    torch = torch_dev
    big = G.workload(1)                 # 100k-stage chain: two hubs of 100k contributions
    small = G.sram_case(16, 24, seed=9)  # shared bitline entries across regions
    say(f"case noalloc: chain {big.n_dev} devices, then sram {small.n_dev} devices, then the chain again")
    cb, tb = setup(torch, big)
    cs_, ts = setup(torch, small)
    xb, xs = tb(big.x), ts(small.x)
    hist = ts(np.random.default_rng(5).standard_normal(4 * small.n_dev))
    Ab0, bb0 = reference(torch, cb, xb)
    As0, bs0 = reference(torch, cs_, xs, hist)
    for what, c, x, h, A0, b0 in (("chain", cb, xb, None, Ab0, bb0), ("sram (smaller)", cs_, xs, hist, As0, bs0),
                                  ("chain again", cb, xb, None, Ab0, bb0)):
        A, b = noalloc(torch, c, x, h)
        assert np.array_equal(bits(A), bits(A0)), f"{what}: A differs from cs_eval_stamp(region)"
        assert np.array_equal(bits(b), bits(b0)), f"{what}: b differs from cs_eval_stamp(region)"


def test_noalloc_graph_replays(torch_dev):
    torch = torch_dev
    circ = G.chain_case(3000, seed=43)
    say(f"case noalloc graph: chain {circ.n_dev} devices, 3 replays")
    c, t = setup(torch, circ)
    x = t(circ.x)
    reference(torch, c, x)              # uploads the region tables
    A = torch.empty(c.nnz, dtype=torch.float64, device=x.device)
    b = torch.empty(c.n_rows, dtype=torch.float64, device=x.device)
    c.eval_stamp_noalloc(x, AG0, A, b)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        c.eval_stamp_noalloc(x, AG0, A, b)
    rng = np.random.default_rng(44)
    for r in range(3):
        xv = circ.x.copy()
        xv[2:circ.n_nodes - 1] = rng.uniform(0.0, 1.0, circ.n_nodes - 3)
        x.copy_(t(xv))
        A.fill_(float("nan"))
        b.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        A0, b0 = reference(torch, c, x)
        assert np.array_equal(bits(A), bits(A0)), f"replay {r}: A"
        assert np.array_equal(bits(b), bits(b0)), f"replay {r}: b"


def test_noalloc_refusals(torch_dev):
    torch = torch_dev
    circ = G.chain_case(500, seed=45)
    c, t = setup(torch, circ)
    x = t(circ.x)
    A = torch.empty(c.nnz, dtype=torch.float64, device=x.device)
    b = torch.empty(c.n_rows, dtype=torch.float64, device=x.device)
    with pytest.raises(CS.CsError) as e:       # no region tables on the device yet
        c.eval_stamp_noalloc(x, AG0, A, b)
    assert e.value.status == -4
    big = G.sram_case(512, 512, seed=7)        # about 26 MB of staged contributions
    say(f"case noalloc refusal: sram {big.n_dev} devices")
    cb, tb = setup(torch, big)
    xb = tb(big.x)
    Ab, bb = reference(torch, cb, xb)
    with pytest.raises(CS.CsError) as e:
        cb.eval_stamp_noalloc(xb, AG0, Ab, bb)
    assert e.value.status == -5 and "bytes of scratch" in str(e.value)
