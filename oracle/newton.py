"""Newton-Raphson loop of the oracle (TEST INFRASTRUCTURE, like the rest of oracle/).

The paper's method sits inside SPICE's Newton iteration (Introduction): at the
present x every device is evaluated and stamped into the linearised MNA system
A x' = b, whose solution x' is the Newton point (b holds A x - F(x), so
x' = x - A^-1 F(x)).  The loop here is the plain form of that iteration with one
safeguard of our own choosing (the paper does not state its damping):

    repeat up to max_iter times:
        A, b = stamp(x)                     serial-order oracle assembly
        y    = solve(A, y = b)              scipy's sparse LU (SuperLU) as the solve
        d    = y - x, node rows clamped to [-vstep, vstep] (branch rows not)
        x    = x + d
        stop when max |d| <= tol

Returns x, the number of solves and max |d| per iteration."""
from __future__ import annotations

import numpy as np

from . import oracle as O


def newton(circ, nmos: dict, pmos: dict, x0=None, ag0: float = 0.0, hist=None, vstep: float = 0.3,
           tol: float = 1e-9, max_iter: int = 100):
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    rp, ci = O.pattern(circ)
    n = circ.n_rows
    n_node = circ.n_nodes - 1
    x = np.array(circ.x if x0 is None else x0, dtype=np.float64, copy=True)
    steps = []
    for it in range(1, max_iter + 1):
        A, b = O.assemble(circ, rp, ci, nmos, pmos, ag0, hist, x=x)
        M = sp.csr_matrix((A, ci, rp), shape=(n, n)).tocsc()
        y = spl.spsolve(M, b)
        d = y - x
        d[:n_node] = np.clip(d[:n_node], -vstep, vstep)
        x = x + d
        steps.append(float(np.max(np.abs(d))) if n else 0.0)
        if not np.isfinite(steps[-1]):
            raise FloatingPointError("Newton step is not finite")
        if steps[-1] <= tol:
            return x, it, steps
    return x, max_iter, steps
