"""Pins of the oracle's model M (the project's BSIM4-core reading; the paper names
BSIM 4.82 without equations) against what the physics and the mathematics fix:

* the stamped conductance matrix Y equals central finite differences of the
  terminal residual f = I + ag0*Q (Methodology: linearised contributions);
* current and charge conservation (Kirchhoff) on every device;
* PMOS at -V is exactly -(NMOS at V); drain/source exchange symmetry;
* closed-form limits (zero body bias, zero drain bias, strong inversion,
  subthreshold slope, long-channel linear region);
* the physically expected direction of every model-card parameter's effect
  (catches a dropped term or a flipped sign);
* the CMOS inverter transfer point;
* values from an independent implementation of the same equations (3 digits).
"""
import math

import numpy as np
import pytest

from paper_2604_03079_amd import netgen as G

NC = G.default_card(1)
PC = G.default_card(-1)


def ev(orc, card, pol, W, L, VTH0, V, ag0=0.0, hist=None, trace=False):
    return orc.device_eval(card, pol, W, L, VTH0, V, ag0, hist, trace)


def random_devices(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        pol = 1 if rng.random() < 0.5 else -1
        W = rng.uniform(0.2e-6, 20e-6)
        L = rng.uniform(45e-9, 500e-9)
        VTH0 = pol * (0.40 + 0.02 * rng.standard_normal())
        V = rng.uniform(0.0, 1.2, 4)
        yield pol, W, L, VTH0, V


def test_independent_reference_values(orc):
    # Same equations evaluated by a separate implementation written when model M
    # was fixed: NMOS, W = 1 um, L = 45 nm, VTH0 = 0.40, vbs = 0.
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 45e-9, 0.40, [1.0, 1.0, 0.0, 0.0], trace=True)
    assert tr["ids"] == pytest.approx(0.943e-3, rel=1.5e-3)
    assert tr["qinv"] == pytest.approx(-4.13e-16, rel=1.5e-3)
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 45e-9, 0.40, [0.5, 0.5, 0.0, 0.0], trace=True)
    assert tr["ids"] == pytest.approx(0.171e-3, rel=3e-3)


@pytest.mark.parametrize("ag0", [0.0, 1e12])
def test_Y_is_the_jacobian_of_the_terminal_residual(orc, ag0):
    eps = 1e-7
    for pol, W, L, VTH0, V in random_devices(300, seed=1 if ag0 else 2):
        card = NC if pol > 0 else PC
        vds = pol * (V[0] - V[2])
        if abs(vds) < 1e-4:
            continue
        Y, _, _, _ = ev(orc, card, pol, W, L, VTH0, V, ag0)
        fd = np.zeros((4, 4))
        for u in range(4):
            Vp = V.copy(); Vp[u] += eps
            Vm = V.copy(); Vm[u] -= eps
            _, _, Ip, Qp = ev(orc, card, pol, W, L, VTH0, Vp, ag0)
            _, _, Im, Qm = ev(orc, card, pol, W, L, VTH0, Vm, ag0)
            fd[:, u] = ((Ip + ag0 * Qp) - (Im + ag0 * Qm)) / (2 * eps)
        scale = np.abs(Y).max() + 1e-30
        assert np.abs(fd - Y).max() <= 1e-6 * scale, (pol, W, L, V, fd, Y)


def test_conservation(orc):
    for pol, W, L, VTH0, V in random_devices(500, seed=3):
        card = NC if pol > 0 else PC
        Y, bl, I, Q = ev(orc, card, pol, W, L, VTH0, V, 1e12)
        assert I.sum() == 0.0 and I[1] == 0.0 and I[3] == 0.0
        assert abs(Q.sum()) <= 8 * np.spacing(np.abs(Q).max())
        sY = np.abs(Y).max()
        assert np.abs(Y.sum(axis=0)).max() <= 16 * np.spacing(sY)   # KCL rows
        assert np.abs(Y.sum(axis=1)).max() <= 16 * np.spacing(sY)   # translation invariance
        assert abs(bl.sum()) <= 1e-13 * (np.abs(bl).max() + np.abs(I).max() + 1e12 * np.abs(Q).max())


def test_local_rhs_definition_and_history(orc):
    for pol, W, L, VTH0, V in random_devices(50, seed=4):
        card = NC if pol > 0 else PC
        ag0 = 1e12
        Y, bl, I, Q = ev(orc, card, pol, W, L, VTH0, V, ag0)
        dv = np.array([V[0] - V[2], V[1] - V[2], 0.0, V[3] - V[2]])
        ref = Y @ dv - I - ag0 * Q
        assert np.allclose(bl, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        hist = np.array([1e-4, -2e-4, 3e-4, -4e-4])
        _, bl2, _, _ = ev(orc, card, pol, W, L, VTH0, V, ag0, hist)
        assert np.allclose(bl2 - bl, hist, rtol=0, atol=1e-15)


def test_pmos_mirror_is_bit_exact(orc):
    for _, W, L, VTH0, V in random_devices(300, seed=5):
        vth = abs(VTH0)
        Yn, bn, In, Qn = ev(orc, NC, 1, W, L, vth, V, 1e12)
        Yp, bp, Ip, Qp = ev(orc, NC, -1, W, L, -vth, -V, 1e12)
        assert np.array_equal(Yp, Yn)
        assert np.array_equal(Ip, -In) and np.array_equal(Qp, -Qn) and np.array_equal(bp, -bn)


def test_drain_source_exchange(orc):
    perm = [2, 1, 0, 3]
    for pol, W, L, VTH0, V in random_devices(300, seed=6):
        card = NC if pol > 0 else PC
        Y, bl, I, Q = ev(orc, card, pol, W, L, VTH0, V, 1e12)
        Ys, bls, Is, Qs = ev(orc, card, pol, W, L, VTH0, V[perm], 1e12)
        assert np.allclose(Is, I[perm], rtol=1e-12, atol=1e-12 * np.abs(I).max() + 1e-30)
        assert np.allclose(Qs, Q[perm], rtol=1e-10, atol=1e-12 * np.abs(Q).max())
        assert np.allclose(Ys, Y[np.ix_(perm, perm)], rtol=1e-10, atol=1e-11 * np.abs(Y).max())


def test_mode_switch_is_continuous(orc):
    # Across vds = 0 the frame swaps drain and source.  Currents, charges and the
    # conductance part of Y (ag0 = 0) are continuous; the capacitance part is not
    # required to be, since charges referenced to the frame's source (body charge,
    # threshold body effect) change reference terminal, as in BSIM4.
    for pol, W, L, VTH0, V in random_devices(100, seed=7):
        card = NC if pol > 0 else PC
        for sgn in (1.0, -1.0):
            Va = V.copy(); Va[0] = Va[2] + sgn * 1e-9
            Vb = V.copy(); Vb[0] = Vb[2] - sgn * 1e-9
            Ya, _, Ia, Qa = ev(orc, card, pol, W, L, VTH0, Va, 0.0)
            Yb, _, Ib, Qb = ev(orc, card, pol, W, L, VTH0, Vb, 0.0)
            assert np.allclose(Ya, Yb, rtol=1e-5, atol=1e-6 * np.abs(Ya).max())
            assert np.allclose(Qa, Qb, rtol=1e-6, atol=1e-6 * np.abs(Qa).max())
            assert np.abs(Ia).max() < 1e-9 and np.abs(Ib).max() < 1e-9


def test_zero_bias_limits(orc):
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 60e-9, 0.4, [0.7, 0.9, 0.0, 0.0], trace=True)
    assert abs(tr["vbseff"]) <= 4 * np.spacing(0.95 * NC["phis"])     # M1 at vbs = 0
    _, _, I, _, tr = ev(orc, NC, 1, 1e-6, 60e-9, 0.4, [0.3, 0.9, 0.3, 0.0], trace=True)
    assert abs(tr["vdseff"]) <= 1e-15 and I[0] == 0.0 or abs(I[0]) < 1e-18
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 60e-9, 0.4, [1e-3, 0.9, 0.0, 0.0], trace=True)
    # small vds: Vdseff -> vds * Vdsat / (Vdsat + DELTA), the slope of the smoothing at 0
    assert tr["vdseff"] == pytest.approx(1e-3 * tr["vdsat"] / (tr["vdsat"] + NC["delta"]), rel=1e-2)
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 60e-9, 0.4, [1.2, 0.9, 0.0, 0.0], trace=True)
    assert tr["vdseff"] == pytest.approx(tr["vdsat"], rel=2e-2)        # saturation: Vdseff ~ Vdsat


def test_strong_inversion_and_subthreshold_limits(orc):
    # strong inversion: Vgsteff -> Vgst
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 1e-6, 0.05, [0.05, 1.2, 0.0, 0.0], trace=True)
    assert tr["vgst"] > 30 * tr["n"] * 0.0258
    assert tr["vgsteff"] == pytest.approx(tr["vgst"], rel=1e-6)
    # subthreshold: d ln(Ids)/d vgs -> 1/(n VT), and Vgsteff -> (nvt/(n COXE KS)) e^((Vgst-VOFF)/nvt)
    VT = 8.617333262e-5 * NC["tnom"]
    _, _, _, _, tr = ev(orc, NC, 1, 1e-6, 1e-6, 0.45, [0.5, 0.0, 0.0, 0.0], trace=True)
    slope = tr["dids"][1] / tr["ids"]
    assert slope == pytest.approx(1.0 / (tr["n"] * VT), rel=2e-2)


def test_long_channel_linear_region_square_law(orc):
    # L = 20 um, vds small: Ids -> (W/L) mu Cox (Vgst vds - Abulk vds^2 / 2)
    W, L, vds = 2e-6, 20e-6, 0.02
    _, _, _, _, tr = ev(orc, NC, 1, W, L, 0.4, [vds, 1.0, 0.0, 0.0], trace=True)
    coxe = 3.9 * 8.8541878128e-12 / NC["toxe"]
    ref = (W / L) * tr["mu"] * coxe * (tr["vgst"] * vds - tr["abulk"] * vds * vds / 2)
    assert tr["ids"] == pytest.approx(ref, rel=0.06)      # 2*VT/Vgst ~ 7e-2 of V2 = Vgst + 2VT
    # SCE and DIBL vanish for long channels
    assert tr["theta_sce"] < 1e-100 and tr["theta_dibl"] < 1e-100


PARAM_SIGNS = [
    # (card field, bias (vd, vg, vs, vb), quantity, expected sign of d quantity / d param)
    ("u0", (0.8, 0.9, 0.0, 0.0), "ids", +1),
    ("ua", (0.8, 0.9, 0.0, 0.0), "ids", -1),
    ("ub", (0.8, 0.9, 0.0, 0.0), "ids", -1),
    ("uc", (0.8, 0.9, 0.0, -0.4), "ids", +1),
    ("vsat", (0.8, 0.9, 0.0, 0.0), "ids", +1),
    ("k1", (0.8, 0.9, 0.0, -0.4), "vth", +1),
    ("k2", (0.8, 0.9, 0.0, -0.4), "vth", +1),
    ("k3", (0.8, 0.9, 0.0, 0.0), "vth", +1),
    ("dvt0", (0.8, 0.9, 0.0, 0.0), "vth", -1),
    ("dvt1", (0.8, 0.9, 0.0, 0.0), "vth", +1),
    ("eta0", (0.8, 0.9, 0.0, 0.0), "vth", -1),
    ("dsub", (0.8, 0.9, 0.0, 0.0), "vth", +1),
    ("nfactor", (0.8, 0.9, 0.0, 0.0), "n", +1),
    ("cdsc", (0.8, 0.9, 0.0, 0.0), "n", +1),
    ("voff", (0.8, 0.2, 0.0, 0.0), "ids", -1),      # subthreshold Ids ~ exp((Vgst - VOFF)/nvt)
    ("a0", (0.9, 0.9, 0.0, 0.0), "abulk", +1),
    ("lambda_l", (1.0, 0.7, 0.0, 0.0), "ids", +1),
    ("delta", (0.3, 0.9, 0.0, 0.0), "vdseff", -1),
    ("delta1", (0.8, 0.9, 0.0, 0.5), "vbseff", -1),   # forward body bias: more smoothing
    ("toxe", (0.8, 0.9, 0.0, 0.0), "ids", -1),
    ("cgdo", (0.2, 0.9, 0.0, 0.0), "qd", -1),
    ("w0", (0.8, 0.9, 0.0, 0.0), "vth", -1),
    ("vbi", (0.8, 0.9, 0.0, 0.0), "vth", -1),
]


@pytest.mark.parametrize("field,V,qty,sign", PARAM_SIGNS)
def test_parameter_effect_direction(orc, field, V, qty, sign):
    W, L, VTH0 = 1e-6, 60e-9, 0.4
    base = dict(NC)
    h = 1e-3 * abs(base[field]) if base[field] != 0 else 1e-6
    up = dict(base); up[field] = base[field] + h
    dn = dict(base); dn[field] = base[field] - h
    qu = ev(orc, up, 1, W, L, VTH0, np.array(V), trace=True)[4][qty]
    qd = ev(orc, dn, 1, W, L, VTH0, np.array(V), trace=True)[4][qty]
    d = (qu - qd) / (2 * h)
    assert np.sign(d) == sign and abs(qu - qd) > 1e-9 * abs(qu), (field, qu, qd)


def test_width_and_vth0_effects(orc):
    V = np.array([0.8, 0.9, 0.0, 0.0])
    i1 = ev(orc, NC, 1, 1e-6, 60e-9, 0.4, V, trace=True)[4]
    i2 = ev(orc, NC, 1, 2e-6, 60e-9, 0.4, V, trace=True)[4]
    assert 1.9 < i2["ids"] / i1["ids"] < 2.1      # ~ linear in W (narrow-width term aside)
    assert i2["cg"] == 2 * i1["cg"]
    i3 = ev(orc, NC, 1, 1e-6, 60e-9, 0.45, V, trace=True)[4]
    assert i3["vth"] - i1["vth"] == pytest.approx(0.05, rel=1e-12)
    assert i3["ids"] < i1["ids"]


def test_inverter_transfer_point(orc):
    sym = G.default_card(-1, symmetric=True)
    vdd = 1.0
    W, L, VTH0 = 1e-6, 60e-9, 0.4
    Vn = np.array([0.5, 0.5, 0.0, 0.0])
    Vp = np.array([0.5, 0.5, vdd, vdd])
    _, _, In, _ = ev(orc, NC, 1, W, L, VTH0, Vn)
    _, _, Ip, _ = ev(orc, sym, -1, W, L, -VTH0, Vp)
    assert In[0] + Ip[0] == 0.0                      # symmetric card: VM = Vdd/2 exactly

    def imbalance(v):
        _, _, a, _ = ev(orc, NC, 1, W, L, VTH0, np.array([v, v, 0.0, 0.0]))
        _, _, b, _ = ev(orc, PC, -1, W, L, -VTH0, np.array([v, v, vdd, vdd]))
        return a[0] + b[0]
    lo, hi = 0.05, 0.95
    assert imbalance(lo) < 0 < imbalance(hi)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if imbalance(mid) < 0:
            lo = mid
        else:
            hi = mid
    assert 0.3 < lo < 0.5                             # weaker PMOS (U0_P < U0_N): VM < Vdd/2


def test_operation_count(orc):
    n = orc.model_opcount(NC, 1, 1e-6, 45e-9, 0.4, [0.7, 0.9, 0.1, 0.0], 1e12)
    assert 700 < n < 1000
    # the size-dependent constants, counted by hand from their formulas (products of
    # card values alone, such as 2 WINT or (K3 TOXE) PHIS, are card constants, not
    # per-device work): Weff, Leff, VTH0i (3); theta_sce and theta_dibl: a product, a
    # quotient, pcosh, a difference and a quotient each (4 + pcosh), pcosh = pexp (the
    # argument's product, rint-free Cody-Waite reduction 4 ops, 13 Horner steps of 2)
    # + 3; vth_s: DVT0 theta_sce, its product with (VBI - PHIS), the difference, Weff +
    # W0, the quotient, the sum (6); beta0, lambda, AbL, Cg, Cov (2 + 1 + 3 + 2 + 1)
    pexp = 5 + 2 * 13
    assert orc.model_sizedep_opcount(NC, 1, 1e-6, 45e-9, 0.4, [0.7, 0.9, 0.1, 0.0], 1e12) == \
        3 + 2 * (4 + pexp + 3) + 6 + (2 + 1 + 3 + 2 + 1)
