"""Full-size parity of the configurations the benchmark reports.

* The 512-circuit sizing batch (256 two-stage op-amps, 192 chains of 100 to 10,000
  stages, 64 rings of 501 to 50,001 stages; 2,388,511 FETs): the schedule chosen by
  the library's autotuner (cs_batch_tune), and the region schedule, reproduce every
  circuit's oracle colour replay bit for bit.
* Its adjoint: the batched VJP of <A_bar, A> + <b_bar, b> (cotangents N(0, 1)) with
  respect to every device's W, L and VTH0 is within 1e-8 of the oracle's
  complex-step gradient, scaled by the device's sum |cotangent * sensitivity| (plus
  8 ulps of its rounding scale, vjpbound), on every one of the 2,388,511 devices; and a directional central difference of the
  GPU forward (step 1e-6 relative in every device at once) agrees with the adjoint
  within 1e-6 of the directional scale.
* The 10,000-stage chain: the same central-difference check (its oracle-gradient
  check is in test_gpu_batch_adjoint)."""
import sys

import numpy as np
import pytest
import vjpbound

from paper_2604_03079_amd import colorstamp as CS
from paper_2604_03079_amd import netgen as G

pytestmark = pytest.mark.gpu
NC, PC = G.default_card(1), G.default_card(-1)
AG0 = 1e12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bits(a):
    return np.ascontiguousarray(a).view(np.int64)


@pytest.fixture(scope="module")
def full_batch(orc):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    say("case full batch: generating 512 circuits and their oracle replays")
    circs = G.workload(3)
    pats = [orc.pattern(c) for c in circs]
    ref = []
    for c, (rp, ci) in zip(circs, pats):
        col, _, _ = orc.colour(c, True)
        ref.append(orc.assemble(c, rp, ci, NC, PC, AG0, col=col, exclude=True))
    B = CS.Batch([CS.prepare(c, True) for c in circs])
    dev = torch.device("cuda:0")
    cat = lambda k: torch.from_numpy(np.concatenate([getattr(c, k) for c in circs])).to(dev)
    say(f"  batch: {B.n_dev} devices, {B.n_rows} rows, {B.nnz} nonzeros")
    return dict(torch=torch, circs=circs, pats=pats, ref=ref, B=B, W=cat("W"), L=cat("L"), V=cat("VTH0"),
                x=cat("x"))


def check_per_circuit(fb, A, b, what):
    B = fb["B"]
    Ah, bh = A.cpu().numpy(), b.cpu().numpy()
    for i, (A0, b0) in enumerate(fb["ref"]):
        assert np.array_equal(bits(Ah[B.nnz_off[i]:B.nnz_off[i + 1]]), bits(A0)), f"{what}: circuit {i} A"
        assert np.array_equal(bits(bh[B.row_off[i]:B.row_off[i + 1]]), bits(b0)), f"{what}: circuit {i} b"


@pytest.mark.timeout(600)
def test_full_batch_tuned_schedule_bit_exact(full_batch):
    fb = full_batch
    torch, B = fb["torch"], fb["B"]
    A = torch.full((B.nnz,), float("nan"), dtype=torch.float64, device="cuda:0")
    b = torch.full((B.n_rows,), float("nan"), dtype=torch.float64, device="cuda:0")
    say("case full batch: cs_batch_tune")
    best = B.tune(fb["W"], fb["L"], fb["V"], fb["x"], AG0, A, b, reps=3)
    say(f"  tuned: {best}")
    assert best["tried"] >= 2 and best["ms"] > 0
    A.fill_(float("nan"))
    b.fill_(float("nan"))
    B.eval_stamp(fb["x"], AG0, None, A, b)
    torch.cuda.synchronize()
    B.check()
    check_per_circuit(fb, A, b, f"tuned {best['schedule']} block {best['block']}")
    for schedule in ("region", "persistent"):
        say(f"case full batch: {schedule} schedule")
        B.set_launch(256, -1, 1024 if schedule == "persistent" else 0, schedule)
        B.set_params(fb["W"], fb["L"], fb["V"])
        A.fill_(float("nan"))
        B.eval_stamp(fb["x"], AG0, None, A, b)
        torch.cuda.synchronize()
        B.check()
        check_per_circuit(fb, A, b, schedule)


@pytest.mark.timeout(900)
def test_full_batch_vjp_every_device_within_1e8(full_batch, orc):
    fb = full_batch
    torch, B, circs = fb["torch"], fb["B"], fb["circs"]
    B.set_launch(256, -1, 0, "region")
    B.set_params(fb["W"], fb["L"], fb["V"])
    Ab, bb = G.cotangents(B.nnz, B.n_rows, seed=50)
    say("case full batch vjp")
    g = B.vjp(fb["x"], AG0, torch.from_numpy(Ab).to("cuda:0"), torch.from_numpy(bb).to("cuda:0"))
    torch.cuda.synchronize()
    g = [v.cpu().numpy() for v in g]
    worst = [0.0, 0.0, 0.0]
    for i, c in enumerate(circs):
        rp, ci = fb["pats"][i]
        Abi = Ab[B.nnz_off[i]:B.nnz_off[i + 1]]
        bbi = bb[B.row_off[i]:B.row_off[i + 1]]
        d0, d1 = B.dev_off[i], B.dev_off[i + 1]
        w = vjpbound.check(orc, [g[k][d0:d1] for k in range(3)], c, rp, ci, NC, PC, AG0, Abi, bbi,
                           label=f"circuit {i} ({c.name})")
        worst = [max(a, b) for a, b in zip(worst, w)]
    say(f"  worst relative error W {worst[0]:.2e} L {worst[1]:.2e} VTH0 {worst[2]:.2e}")


def directional_fd(torch, set_params, forward, Ab, bb, base, g, seed):
    """Central difference of J = <Ab, A> + <bb, b> along a random direction in each
    parameter (step 1e-6 relative, every device at once) against the adjoint's
    directional derivative; returns (fd, adjoint, scale) per parameter."""
    rng = np.random.default_rng(seed)
    out = []
    for k, name in enumerate(("W", "L", "V")):
        d = rng.standard_normal(base[name].shape[0])
        h = 1e-6 * np.abs(base[name]) * d
        vals = []
        for sgn in (1.0, -1.0):
            p = {kk: v for kk, v in base.items()}
            p[name] = base[name] + sgn * h
            set_params(*(torch.from_numpy(np.ascontiguousarray(p[kk])).to("cuda:0") for kk in ("W", "L", "V")))
            A, b = forward()
            vals.append(float(torch.dot(Ab, A)) + float(torch.dot(bb, b)))
        fd = (vals[0] - vals[1]) / 2.0
        an = float(np.sum(g[k] * h))
        scale = float(np.sum(np.abs(g[k] * h)))
        out.append((name, fd, an, scale))
    return out


@pytest.mark.timeout(600)
def test_full_batch_central_differences(full_batch):
    fb = full_batch
    torch, B = fb["torch"], fb["B"]
    B.set_launch(256, -1, 0, "region")
    B.set_params(fb["W"], fb["L"], fb["V"])
    Ab, bb = G.cotangents(B.nnz, B.n_rows, seed=50)
    Abd, bbd = torch.from_numpy(Ab).to("cuda:0"), torch.from_numpy(bb).to("cuda:0")
    g = [v.cpu().numpy() for v in B.vjp(fb["x"], AG0, Abd, bbd)]
    A = torch.empty(B.nnz, dtype=torch.float64, device="cuda:0")
    b = torch.empty(B.n_rows, dtype=torch.float64, device="cuda:0")

    def forward():
        B.eval_stamp(fb["x"], AG0, None, A, b)
        torch.cuda.synchronize()
        return A, b

    base = dict(W=fb["W"].cpu().numpy(), L=fb["L"].cpu().numpy(), V=fb["V"].cpu().numpy())
    for name, fd, an, scale in directional_fd(torch, B.set_params, forward, Abd, bbd, base, g, 12):
        say(f"case full batch fd {name}: fd={fd:.9e} adjoint={an:.9e} scale={scale:.3e} "
            f"rel={abs(fd - an) / scale:.2e}")
        assert abs(fd - an) <= 1e-6 * scale
    B.set_params(fb["W"], fb["L"], fb["V"])


@pytest.mark.timeout(300)
def test_chain10k_central_differences(orc):
    import torch
    circ = G.workload(4)
    c = CS.prepare(circ, True)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    c.set_params(t(circ.W), t(circ.L), t(circ.VTH0))
    x = t(circ.x)
    Ab, bb = G.cotangents(c.nnz, c.n_rows, seed=50)
    Abd, bbd = t(Ab), t(bb)
    g = [v.cpu().numpy() for v in c.vjp(x, AG0, Abd, bbd)]
    A = torch.empty(c.nnz, dtype=torch.float64, device=dev)
    b = torch.empty(c.n_rows, dtype=torch.float64, device=dev)

    def forward():
        c.eval_stamp(x, AG0, None, A, b, "region")
        torch.cuda.synchronize()
        return A, b

    base = dict(W=circ.W, L=circ.L, V=circ.VTH0)
    for name, fd, an, scale in directional_fd(torch, c.set_params, forward, Abd, bbd, base, g, 13):
        say(f"case chain10k fd {name}: fd={fd:.9e} adjoint={an:.9e} rel={abs(fd - an) / scale:.2e}")
        assert abs(fd - an) <= 1e-6 * scale
