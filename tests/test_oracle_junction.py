"""Pins of the oracle's second model level: model M plus the source/drain-body
junctions of BSIM4 (card jmod = 1), the fuller subset the kernels evaluate behind
the same interface.

* Diode current against the closed form Is (e^(v / (nj VT)) - 1), Is = js Weff hdif,
  for both junctions with the channel cut off, and the tangent continuation above
  vjmax (value and slope continuous there).
* Depletion charge of an abrupt junction against its closed forms below and above
  fc pb (the SPICE linear-capacitance continuation), the capacitance equal to dQ/dv
  on both sides and continuous at fc pb.
* With junctions on, Y is still the Jacobian of I + ag0 Q (central differences),
  currents and charges are conserved, and the PMOS mirror is bit-exact.
* jmod = 0 leaves model M's outputs bit for bit unchanged."""
import math

import numpy as np
import pytest

from paper_2604_03079_amd import netgen as G

NJ, PJ = G.junction_card(1), G.junction_card(-1)
NC, PC = G.default_card(1), G.default_card(-1)
KB_Q = 8.617333262e-5
VT = KB_Q * NJ["tnom"]


def ev(orc, card, pol, W, V, ag0=0.0, L=60e-9, VTH0=None):
    return orc.device_eval(card, pol, W, L, pol * 5.0 if VTH0 is None else VTH0, np.asarray(V, float), ag0)


def diode(v, Is, c=NJ):
    nvt = c["nj"] * VT
    if v <= c["vjmax"]:
        return Is * math.expm1(max(v / nvt, -40.0))
    el = math.exp(c["vjmax"] / nvt)
    return Is * (el - 1.0) + Is * el / nvt * (v - c["vjmax"])


def depletion(v, Cj0, c=NJ):
    pb, fc = c["pb"], c["fc"]
    if v < fc * pb:
        return 2 * pb * Cj0 * (1 - math.sqrt(1 - v / pb))
    F1 = 2 * pb * (1 - (1 - fc) ** 0.5)
    F2 = (1 - fc) ** 1.5
    F3 = 1 - 1.5 * fc
    return Cj0 * (F1 + (F3 * (v - fc * pb) + (v * v - (fc * pb) ** 2) / (4 * pb)) / F2)


@pytest.mark.parametrize("vbd,vbs", [(0.6, 0.3), (0.2, -0.5), (-1.0, 0.45), (0.75, 0.7), (1.1, -2.0), (0.9, -3.0)])
def test_diode_currents_closed_form(orc, vbd, vbs):
    W = 2e-6
    Is = NJ["js"] * W * NJ["hdif"]
    Vb = 1.5
    V = [Vb - vbd, 0.0, Vb - vbs, Vb]          # gate at 0, VTH0 = 5 V: channel cut off
    _, _, I, _ = ev(orc, NJ, 1, W, V)
    _, _, I0, _ = ev(orc, NC, 1, W, V)
    jd, js_ = diode(vbd, Is), diode(vbs, Is)
    assert I[3] == pytest.approx(jd + js_, rel=1e-12, abs=1e-30)
    assert (I0[0] - I[0]) == pytest.approx(jd, rel=1e-12, abs=1e-30)
    assert (I0[2] - I[2]) == pytest.approx(js_, rel=1e-12, abs=1e-30)
    # PMOS: the same junctions with every voltage and current mirrored
    _, _, Ip, _ = ev(orc, PJ, -1, W, [-v for v in V])
    assert Ip[3] == pytest.approx(-(jd + js_), rel=1e-12, abs=1e-30)


def test_diode_continuation_is_continuous(orc):
    W = 1e-6
    Is = NJ["js"] * W * NJ["hdif"]
    nvt = NJ["nj"] * VT
    v0, h = NJ["vjmax"], 1e-7
    I = []
    for v in (v0 - 2 * h, v0 - h, v0 + h, v0 + 2 * h):
        _, _, Iv, _ = ev(orc, NJ, 1, W, [0.0, 0.0, 0.0, v])      # both junctions at v
        I.append(Iv[3] / 2)
    g_below, g_above = (I[1] - I[0]) / h, (I[3] - I[2]) / h
    g0 = Is * math.exp(v0 / nvt) / nvt
    assert g_below == pytest.approx(g0, rel=1e-4) and g_above == pytest.approx(g0, rel=1e-4)
    assert (I[1] + I[2]) / 2 == pytest.approx(Is * math.expm1(v0 / nvt), rel=1e-6)


@pytest.mark.parametrize("v", [-3.0, -0.4, 0.0, 0.3, 0.5, 0.8, 1.2])
def test_depletion_charge_closed_form_and_capacitance(orc, v):
    W = 3e-6
    Cj0 = NJ["cj"] * W * NJ["hdif"]
    V = [1.0 - v, 0.0, 1.0 + 2.0, 1.0]      # drain junction at v, source junction reverse 2 V
    _, _, _, Q = ev(orc, NJ, 1, W, V)
    _, _, _, Q0 = ev(orc, NC, 1, W, V)
    assert (Q0[0] - Q[0]) == pytest.approx(depletion(v, Cj0), rel=1e-12, abs=1e-35)
    # C = dQ/dv: the capacitance part of Ydd at ag0 = 1 (diode part taken off at ag0 = 0)
    h = 1e-6
    c_fd = (depletion(v + h, Cj0) - depletion(v - h, Cj0)) / (2 * h)
    Y1, _, _, _ = ev(orc, NJ, 1, W, V, ag0=1.0)
    Y0, _, _, _ = ev(orc, NJ, 1, W, V, ag0=0.0)
    Yc1, _, _, _ = ev(orc, NC, 1, W, V, ag0=1.0)
    Yc0, _, _, _ = ev(orc, NC, 1, W, V, ag0=0.0)
    c_model = (Y1[0, 0] - Y0[0, 0]) - (Yc1[0, 0] - Yc0[0, 0])
    assert c_model == pytest.approx(c_fd, rel=1e-6)


def test_capacitance_is_continuous_at_fc_pb(orc):
    W = 1e-6
    v0 = NJ["fc"] * NJ["pb"]
    caps = []
    for v in (v0 - 1e-10, v0 + 1e-10):
        Y1, _, _, _ = ev(orc, NJ, 1, W, [0.0, 0.0, 0.0, v], ag0=1.0)
        Y0, _, _, _ = ev(orc, NJ, 1, W, [0.0, 0.0, 0.0, v], ag0=0.0)
        caps.append(Y1[3, 3] - Y0[3, 3])
    assert caps[0] == pytest.approx(caps[1], rel=1e-8)


def devices(n, seed):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        pol = 1 if rng.random() < 0.5 else -1
        yield (pol, rng.uniform(0.2e-6, 20e-6), rng.uniform(45e-9, 500e-9),
               pol * (0.40 + 0.02 * rng.standard_normal()), rng.uniform(-0.3, 1.3, 4))


@pytest.mark.parametrize("ag0", [0.0, 1e12])
def test_Y_is_the_jacobian_with_junctions(orc, ag0):
    eps = 1e-7
    for pol, W, L, VTH0, V in devices(200, 11 if ag0 else 12):
        card = NJ if pol > 0 else PJ
        if abs(V[0] - V[2]) < 1e-4:
            continue
        Y, _, I, Q = orc.device_eval(card, pol, W, L, VTH0, V, ag0)
        floor = 4 * np.finfo(float).eps * (np.abs(I).max() + ag0 * np.abs(Q).max()) / eps   # difference rounding
        fd = np.zeros((4, 4))
        for u in range(4):
            Vp = V.copy(); Vp[u] += eps
            Vm = V.copy(); Vm[u] -= eps
            _, _, Ip, Qp = orc.device_eval(card, pol, W, L, VTH0, Vp, ag0)
            _, _, Im, Qm = orc.device_eval(card, pol, W, L, VTH0, Vm, ag0)
            fd[:, u] = ((Ip + ag0 * Qp) - (Im + ag0 * Qm)) / (2 * eps)
        assert np.abs(fd - Y).max() <= 1e-6 * np.abs(Y).max() + floor


def test_conservation_and_mirror_with_junctions(orc):
    for pol, W, L, VTH0, V in devices(300, 13):
        card = NJ if pol > 0 else PJ
        Y, bl, I, Q = orc.device_eval(card, pol, W, L, VTH0, V, 1e12)
        assert abs(I.sum()) <= 8 * np.spacing(np.abs(I).max()) and I[1] == 0.0
        assert abs(Q.sum()) <= 8 * np.spacing(np.abs(Q).max())
        sY = np.abs(Y).max()
        assert np.abs(Y.sum(axis=0)).max() <= 16 * np.spacing(sY)
        vth = abs(VTH0)
        Yn, bn, In, Qn = orc.device_eval(NJ, 1, W, L, vth, V, 1e12)
        Yp, bp, Ip, Qp = orc.device_eval(NJ, -1, W, L, -vth, -V, 1e12)
        assert np.array_equal(Yp, Yn) and np.array_equal(Ip, -In) and np.array_equal(Qp, -Qn)
        assert np.array_equal(bp, -bn)


def test_jmod_zero_is_model_m(orc):
    off = dict(NJ, jmod=0.0)
    for pol, W, L, VTH0, V in devices(50, 14):
        a = orc.device_eval(off if pol > 0 else dict(PJ, jmod=0.0), pol, W, L, VTH0, V, 1e12)
        b = orc.device_eval(NC if pol > 0 else PC, pol, W, L, VTH0, V, 1e12)
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
