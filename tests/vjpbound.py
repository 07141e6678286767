"""The bound for a gradient compared with the oracle's complex-step gradient.

Per device and parameter: 1e-8 of the sensitivity scale (sum of |cotangent *
sensitivity| over the device's stamped entries, or_vjp_magnitude), plus 8 ulps of
the device's rounding scale (its largest |cotangent| times the sum of |sensitivity|
over all its local outputs, or_vjp_round_scale).  The second term matters only
where a gradient sits at rounding level beside large local sensitivities: the
source row and column are negated sums of the others and the RHS adds Y (V - V_s)
to the currents and charges, so there the oracle's own value is decided by how
those sums round, and a gradient formed in another order (or from contracted
directions) agrees with it only to that scale."""
import numpy as np

EPS = 2.0 ** -52
REL = 1e-8
ULPS = 8.0


def check(orc, got, circ, rp, ci, nmos, pmos, ag0, Ab, bb, hist=None, ref=None, label=""):
    """Assert got (W, L, VTH0 gradients of circ's devices) within the bound; returns
    the worst |got - ref| / sensitivity scale per parameter."""
    if ref is None:
        ref = orc.vjp(circ, rp, ci, nmos, pmos, ag0, Ab, bb, hist=hist)
    mag = orc.vjp(circ, rp, ci, nmos, pmos, ag0, Ab, bb, hist=hist, magnitude=True)
    scale = None
    worst = []
    for k, what in enumerate(("W", "L", "VTH0")):
        g = np.asarray(got[k])
        d = np.abs(g - ref[k])
        ok = d <= REL * mag[k] + 1e-300
        if not ok.all():
            if scale is None:
                scale = orc.vjp(circ, rp, ci, nmos, pmos, ag0, Ab, bb, hist=hist, magnitude="round")
            ok = d <= REL * mag[k] + ULPS * EPS * scale[k] + 1e-300
        err = d / (mag[k] + 1e-300)
        bad = np.nonzero(~ok)[0]
        assert bad.size == 0, (f"{label} {what}: devices {bad[:8].tolist()} beyond the bound, "
                               f"worst |d|/scale {float(err.max()):.3e}")
        worst.append(float(err.max()) if err.size else 0.0)
    return worst
