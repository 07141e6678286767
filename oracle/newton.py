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

Returns x, the number of solves and max |d| per iteration.

transient() chains backward-Euler steps: before each, the history term of every
device terminal is ag0 times its charge at the present point (the charge current
being ag0 (Q(x) - Q(x_prev)), ag0 = 1/h), then the Newton loop with that ag0."""
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


def history(circ, nmos: dict, pmos: dict, x, ag0: float):
    """ag0 * Q of every device terminal at x, (n_dev, 4)."""
    hist = np.zeros((circ.n_dev, 4))
    for v in range(circ.n_dev):
        t = circ.term[v]
        V = np.array([0.0 if n == 0 else x[n - 1] for n in t])
        pol = int(circ.pol[v])
        _, _, _, Q = O.device_eval(nmos if pol > 0 else pmos, pol, circ.W[v], circ.L[v], circ.VTH0[v], V, 0.0)
        hist[v] = ag0 * Q
    return hist


def transient(circ, nmos: dict, pmos: dict, h: float, n_steps: int, x0=None, **kw):
    """Backward-Euler steps of size h from x0: the iterates after every step (the
    start first) and the Newton iteration counts."""
    ag0 = 1.0 / h
    x = np.array(circ.x if x0 is None else x0, dtype=np.float64, copy=True)
    out, iters = [x.copy()], []
    for _ in range(n_steps):
        hist = history(circ, nmos, pmos, x, ag0)
        x, it, steps = newton(circ, nmos, pmos, x, ag0, hist, **kw)
        if steps[-1] > kw.get("tol", 1e-9):
            raise FloatingPointError("Newton did not converge")
        iters.append(it)
        out.append(x.copy())
    return np.array(out), iters
