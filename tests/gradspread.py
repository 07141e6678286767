"""How well the oracle's gradient is determined, device by device.

Complex steps of different sizes are each an exact derivative of the same rounded
program up to O(h^2); where two of them disagree, the derivative itself is decided
by rounding (a sensitivity formed by cancellation), and no evaluation order can be
expected to agree with another beyond that spread.  Used by the CPU test that names
such devices."""
import numpy as np

STEPS = (1e-20, 3.7e-23, 1.3e-17)


def spread(orc, circ, rp, ci, Ab, bb, nmos, pmos, ag0=1e12):
    """(3, n_dev): per parameter (W, L, VTH0) and device, the largest difference of the
    cotangent-weighted gradient between complex steps of relative size STEPS, over
    the device's scale sum |cotangent * sensitivity|."""
    out = np.zeros((3, circ.n_dev))

    def slot(r, c):
        lo, hi = int(rp[r]), int(rp[r + 1])
        return lo + int(np.searchsorted(ci[lo:hi], c))

    for v in range(circ.n_dev):
        t4 = [int(n) for n in circ.term[v]]
        V = np.array([0.0 if n == 0 else circ.x[n - 1] for n in t4])
        cd = nmos if circ.pol[v] > 0 else pmos
        for which in range(3):
            gs = []
            for h in STEPS:
                dY, dbl = orc.device_dparam(cd, int(circ.pol[v]), circ.W[v], circ.L[v], circ.VTH0[v], V, ag0, None,
                                            which, rel_h=h)
                g = m = 0.0
                for t in range(4):
                    if t4[t] == 0:
                        continue
                    for u in range(4):
                        if t4[u] == 0:
                            continue
                        term = Ab[slot(t4[t] - 1, t4[u] - 1)] * dY[t, u]
                        g += term
                        m += abs(term)
                    term = bb[t4[t] - 1] * dbl[t]
                    g += term
                    m += abs(term)
                gs.append((g, m))
            out[which, v] = max(abs(g - gs[0][0]) for g, _ in gs[1:]) / (gs[0][1] + 1e-300)
    return out
