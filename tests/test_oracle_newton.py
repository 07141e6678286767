"""Pins of the oracle's Newton loop (the iteration around the stamp phase,
Introduction: evaluate, stamp, solve, update until the step vanishes).

* A symmetric inverter chain (PMOS card with the NMOS mobility, equal sizes,
  threshold +-0.4 V) whose input is held at Vdd/2 has every node at exactly Vdd/2:
  the loop reaches it from a random start.  That point is metastable (each stage
  amplifies a rounding residue by its gain, about 35 here), so the chain is short.
* With the input at 0 V the stages settle at the rails, alternately, and the KCL
  residual built from device currents alone vanishes at the result.
* A resistor divider (linear) is solved by the first step: the second step is zero
  and the voltages are the closed form.
* The last steps contract quadratically (Newton's rate), which fails for a wrong
  Jacobian.
* A backward-Euler step (ag0, history terms) converges to a point where
  I + ag0*Q - hist sums to zero at every node.
* Backward-Euler transients (history = ag0 * Q at the previous point): an inverter
  discharges its output monotonically toward the DC point, and a chain ends at its
  DC operating point."""
import numpy as np
import pytest

from oracle import newton as N
from paper_2604_03079_amd import netgen as G

NC, PC = G.default_card(1), G.default_card(-1)


def kcl(orc, circ, x, ag0=0.0, hist=None):
    """Node residual from device (and resistor) currents only."""
    F = np.zeros(circ.n_nodes - 1)
    for v in range(circ.n_dev):
        t = circ.term[v]
        V = np.array([0.0 if n == 0 else x[n - 1] for n in t])
        _, _, I, Q = orc.device_eval(NC if circ.pol[v] > 0 else PC, int(circ.pol[v]), circ.W[v], circ.L[v],
                                     circ.VTH0[v], V, ag0, None if hist is None else hist[v])
        for k in range(4):
            if t[k] != 0:
                F[t[k] - 1] += I[k] + ag0 * Q[k] - (0.0 if hist is None else hist[v][k])
    # source branch currents enter the node rows of their terminals
    nb = circ.n_nodes - 1
    for j, (p, q) in enumerate(circ.vsrc):
        if p:
            F[p - 1] += x[nb + j]
        if q:
            F[q - 1] -= x[nb + j]
    return F


def test_symmetric_chain_at_half_supply(orc):
    circ = G.drive(G.inverter_chain(2), 2, 0.5)
    n = circ.n_dev
    circ.W, circ.L = np.full(n, 1e-6), np.full(n, 60e-9)
    circ.VTH0 = 0.4 * circ.pol.astype(np.float64)
    rng = np.random.default_rng(3)
    x0 = np.zeros(circ.n_rows)
    x0[:circ.n_nodes - 1] = rng.uniform(0, 1, circ.n_nodes - 1)
    x, it, steps = N.newton(circ, NC, G.default_card(-1, symmetric=True), x0)
    assert steps[-1] <= 1e-9 and it < 60
    assert np.all(np.abs(x[:circ.n_nodes - 1] - np.r_[1.0, np.full(circ.n_nodes - 2, 0.5)]) <= 1e-12)


def test_chain_settles_at_alternating_rails(orc):
    circ = G.chain_dc_case(9, seed=5, vin=0.0)
    x, it, steps = N.newton(circ, NC, PC)
    assert steps[-1] <= 1e-9
    out = x[2:circ.n_nodes - 1]                 # rows of nodes 3.. (stage outputs)
    assert np.all(np.abs(out[0::2] - 1.0) < 1e-3) and np.all(np.abs(out[1::2]) < 1e-3)
    F = kcl(orc, circ, x)
    scale = max(abs(F).max(), 1e-6)             # the largest device current sets the scale
    assert np.all(np.abs(F) <= 1e-9 * scale + 1e-15)
    assert x[circ.n_nodes - 1] < 0              # the supply delivers current (into pos: negative)


def test_linear_divider_is_solved_in_one_step(orc):
    R = np.array([1.0, 2.0, 3.0, 5.0])
    k = R.size
    nodes = [1] + list(range(2, k + 1)) + [0]
    circ = G.Circuit("divider", k + 1, np.zeros((0, 4), np.int32), np.zeros(0, np.int8),
                     np.array([[1, 0]], np.int32), np.array([1.5]), np.zeros(k + 1, np.uint8), 1.5,
                     res=np.array([(nodes[i], nodes[i + 1]) for i in range(k)], np.int32), res_g=1.0 / R)
    circ.W = circ.L = circ.VTH0 = np.zeros(0)
    circ.x = np.zeros(circ.n_rows)
    x, it, steps = N.newton(circ, NC, PC, vstep=10.0)
    assert it == 2 and steps[1] <= 1e-15
    below = np.cumsum(R[::-1])[::-1]
    assert np.allclose(x[:k], 1.5 * below / R.sum(), rtol=1e-15, atol=0)


def test_quadratic_convergence(orc):
    circ = G.chain_dc_case(40, seed=6, vin=0.0)
    x, it, steps = N.newton(circ, NC, PC, tol=1e-14)
    # the last unclamped steps: e_{k+1} <= C e_k^2 with a modest C, until rounding
    e = [s for s in steps if s < 0.3]
    pairs = [(a, b) for a, b in zip(e, e[1:]) if a < 1e-2 and b > 1e-13]
    assert pairs, e
    assert all(b <= 50.0 * a * a for a, b in pairs), pairs


@pytest.mark.parametrize("seed", [7, 8])
def test_backward_euler_step(orc, seed):
    circ = G.chain_dc_case(15, seed=seed, vin=0.3)
    hist = np.random.default_rng(seed).normal(0, 1e-5, (circ.n_dev, 4))
    x, it, steps = N.newton(circ, NC, PC, ag0=1e12, hist=hist)
    assert steps[-1] <= 1e-9
    F = kcl(orc, circ, x, 1e12, hist)
    assert np.all(np.abs(F) <= 1e-9 * max(abs(F).max(), 1e-6) + 1e-15)


def test_transient_discharge_is_monotone_and_settles(orc):
    # one inverter, input held at Vdd, output starting at Vdd: the NMOS discharges the
    # output (through its own charge); backward Euler decreases it step by step toward
    # the DC point, without overshoot
    circ = G.drive(G.inverter_chain(1), 2, 1.0)
    circ = G.draw_params(circ, np.random.default_rng(4), G.W_CHAIN, G.L_CHAIN)
    x0 = np.zeros(circ.n_rows)
    x0[0], x0[1], x0[2] = 1.0, 1.0, 1.0           # vdd, input, output
    xdc, _, _ = N.newton(circ, NC, PC, x0)
    wave, iters = N.transient(circ, NC, PC, 1e-13, 200, x0)
    out = wave[:, 2]
    above = out - xdc[2] > 1e-6
    assert above[:20].all()                       # the decay spans many steps
    assert np.all(np.diff(out)[above[:-1]] < 0)   # strictly falling while above the DC point
    assert np.all(out >= xdc[2] - 1e-9)           # no overshoot
    assert abs(out[-1] - xdc[2]) < 1e-6


def test_transient_reaches_the_dc_point(orc):
    circ = G.chain_dc_case(4, seed=9, vin=0.0)
    xdc, _, steps = N.newton(circ, NC, PC)
    assert steps[-1] <= 1e-9
    wave, iters = N.transient(circ, NC, PC, 5e-12, 400)
    n = circ.n_nodes - 1
    assert np.abs(wave[-1][:n] - xdc[:n]).max() < 1e-6
    assert max(iters) < 30
