"""ctypes binding of the C oracle (TEST INFRASTRUCTURE: only the tests, the smoke
check and the benchmark's CPU-baseline leg load it; the GPU library never does).

Inputs are numpy arrays or the circuit objects of the seeded generators; the
oracle never sees anything produced by the GPU path."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

CARD_FIELDS = ("tnom", "toxe", "ndep", "phis", "vbi", "k1", "k2", "k3", "w0", "dvt0", "dvt1",
               "dsub", "eta0", "nfactor", "cdsc", "voff", "u0", "ua", "ub", "uc", "vsat", "a0",
               "xj", "delta", "delta1", "lambda_l", "cgdo", "lint", "wint",
               "jmod", "js", "nj", "cj", "pb", "fc", "hdif", "vjmax")


class OrCard(C.Structure):
    _fields_ = [(f, C.c_double) for f in CARD_FIELDS]


class OrTrace(C.Structure):
    _fields_ = [("mode", C.c_int), ("x1", C.c_double), ("x2", C.c_double), ("x3", C.c_double)] + [
        (f, C.c_double) for f in (
            "theta_sce", "theta_dibl", "vth_s", "beta0", "lambda_", "abl", "cg", "cov",
            "vbseff", "sqps", "vth", "n", "vgst", "vgsteff", "mu", "esatl", "abulk", "v2",
            "vdsat", "vdseff", "ids0", "ids", "vdc", "vdcv", "qinv", "qb", "qd", "qs", "qg")
    ] + [("dids", C.c_double * 3)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _b  # noqa: WPS433
            _b.build()
        _lib = C.CDLL(_LIB_PATH)
        d, i32, i64, p = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        for name in ("or_pexp", "or_plog1p", "or_softplus", "or_sigma", "or_pcosh"):
            getattr(_lib, name).restype = d
            getattr(_lib, name).argtypes = [d]
        _lib.or_ops.restype = C.c_longlong
        _lib.or_sizedep_ops.restype = C.c_longlong
        _lib.or_count_ops.argtypes = [C.c_int]
        _lib.or_device_eval.argtypes = [p, C.c_int, d, d, d, p, d, p, p, p, p, p, p]
        _lib.or_colour.argtypes = [i32, i32, p, p, p, p, p]
        _lib.or_colour_order.argtypes = [i32, i32, p, p, C.c_int, p, p, p]
        _lib.or_pattern.argtypes = [i32, i32, p, i32, p, i32, p, p, p, p]
        _lib.or_linear_stamp.argtypes = [i32, i32, p, p, p, p, i64, p, p, C.c_int]
        _lib.or_stamp_map.argtypes = [i32, i32, p, p, p, p, p, p, p, p, p]
        _lib.or_assemble.argtypes = [i32, i32, p, p, i32, p, p, i32, p, p, p, p, p, p, p, p, p, p, p, p,
                                     d, p, p, p]
        _lib.or_assemble_omp.argtypes = _lib.or_assemble.argtypes
        _lib.or_omp_threads.restype = C.c_int
        _lib.or_hubsum.restype = d
        _lib.or_hubsum.argtypes = [p, i64]
        _lib.or_vjp.argtypes = [i32, i32, p, p, p, p, p, p, p, p, p, p, d, p, p, p, p, p, p]
        _lib.or_vjp_magnitude.argtypes = [i32, i32, p, p, p, p, p, p, p, p, p, p, d, p, p, p, p, p, p]
        _lib.or_vjp_round_scale.argtypes = [i32, i32, p, p, p, p, p, p, p, p, p, p, d, p, p, p, p, p, p]
        _lib.or_device_dparam.argtypes = [p, C.c_int, d, d, d, p, d, p, C.c_int, p, p]
        _lib.or_device_dparam_h.argtypes = [p, C.c_int, d, d, d, p, d, p, C.c_int, d, p, p]
        _lib.or_elem_array.argtypes = [C.c_int, p, p, i64]
        _lib.or_assemble_magnitude.argtypes = [i32, i32, p, p, i32, p, p, i32, p, p, p, p, p, p, p, p,
                                               p, p, d, p, p, p]
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def card(d: dict) -> OrCard:
    return OrCard(*[float(d[f]) for f in CARD_FIELDS])


def pexp(a: float) -> float:
    return lib().or_pexp(float(a))


def plog1p(y: float) -> float:
    return lib().or_plog1p(float(y))


def softplus(t: float) -> float:
    return lib().or_softplus(float(t))


def sigma(t: float) -> float:
    return lib().or_sigma(float(t))


def pcosh(u: float) -> float:
    return lib().or_pcosh(float(u))


ELEM_KINDS = {"pexp": 0, "plog1p": 1, "softplus": 2, "sigma": 3, "pcosh": 4}


def elem_array(kind: str, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty_like(x)
    lib().or_elem_array(ELEM_KINDS[kind], _ptr(x), _ptr(y), x.shape[0])
    return y


def device_eval(cd: dict, pol: int, W: float, L: float, VTH0: float, V, ag0: float = 0.0,
                hist=None, trace: bool = False):
    """One device.  Returns (Y[4,4], bl[4], I[4], Q[4]) and, with trace=True, the
    intermediate values as a dict."""
    c = card(cd)
    V = np.ascontiguousarray(V, dtype=np.float64)
    h = None if hist is None else np.ascontiguousarray(hist, dtype=np.float64)
    Y = np.zeros(16); bl = np.zeros(4); I = np.zeros(4); Q = np.zeros(4)
    tr = OrTrace()
    lib().or_device_eval(C.byref(c), int(pol), float(W), float(L), float(VTH0), _ptr(V),
                         float(ag0), _ptr(h), _ptr(Y), _ptr(bl), _ptr(I), _ptr(Q),
                         C.byref(tr) if trace else None)
    out = (Y.reshape(4, 4), bl, I, Q)
    if trace:
        d = {f[0]: getattr(tr, f[0]) for f in OrTrace._fields_ if f[0] != "dids"}
        d["dids"] = np.array(tr.dids[:])
        d["lambda"] = d.pop("lambda_")
        return out + (d,)
    return out


def device_dparam(cd: dict, pol: int, W, L, VTH0, V, ag0=0.0, hist=None, which=0, rel_h=None):
    """Complex-step d(Y, bl)/d(theta) of one device (relative step 1e-20 by default)."""
    c = card(cd)
    V = np.ascontiguousarray(V, dtype=np.float64)
    h = None if hist is None else np.ascontiguousarray(hist, dtype=np.float64)
    dY = np.zeros(16); dbl = np.zeros(4)
    if rel_h is None:
        lib().or_device_dparam(C.byref(c), int(pol), float(W), float(L), float(VTH0), _ptr(V),
                               float(ag0), _ptr(h), int(which), _ptr(dY), _ptr(dbl))
    else:
        lib().or_device_dparam_h(C.byref(c), int(pol), float(W), float(L), float(VTH0), _ptr(V),
                                 float(ag0), _ptr(h), int(which), float(rel_h), _ptr(dY), _ptr(dbl))
    return dY.reshape(4, 4), dbl


def model_opcount(cd: dict, pol: int, W, L, VTH0, V, ag0=1e12, hist=None) -> int:
    """FP64 operations (+, -, *, /, sqrt) of one model-M evaluation."""
    lib().or_count_ops(1)
    device_eval(cd, pol, W, L, VTH0, V, ag0, hist)
    n = lib().or_ops()
    lib().or_count_ops(0)
    return int(n)


def model_sizedep_opcount(cd: dict, pol: int, W, L, VTH0, V, ag0=1e12, hist=None) -> int:
    """The share of model_opcount spent on the size-dependent constants (W, L, VTH0
    only), which a simulator computes once per parameter set."""
    lib().or_count_ops(1)
    device_eval(cd, pol, W, L, VTH0, V, ag0, hist)
    n = lib().or_sizedep_ops()
    lib().or_count_ops(0)
    return int(n)


def colour(circ, exclude: bool):
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    excl = np.ascontiguousarray(circ.exclude, dtype=np.uint8) if exclude else None
    col = np.zeros(circ.n_dev, dtype=np.int32)
    nc = C.c_int32(0)
    ne = C.c_int64(0)
    rc = lib().or_colour(circ.n_nodes, circ.n_dev, _ptr(term), _ptr(excl), _ptr(col),
                         C.byref(nc), C.byref(ne))
    if rc != 0:
        raise RuntimeError(f"or_colour failed: {rc}")
    return col, int(nc.value), int(ne.value)


ORDERS = {"natural": 0, "largest_first": 1, "dsatur": 2}


def colour_order(circ, exclude: bool, order: str):
    """Greedy colouring in another vertex order (largest first, DSATUR)."""
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    excl = np.ascontiguousarray(circ.exclude, dtype=np.uint8) if exclude else None
    col = np.zeros(circ.n_dev, dtype=np.int32)
    nc = C.c_int32(0)
    ne = C.c_int64(0)
    rc = lib().or_colour_order(circ.n_nodes, circ.n_dev, _ptr(term), _ptr(excl), ORDERS[order], _ptr(col),
                               C.byref(nc), C.byref(ne))
    if rc != 0:
        raise RuntimeError(f"or_colour_order failed: {rc}")
    return col, int(nc.value), int(ne.value)


def _resistors(circ):
    """Series resistors of a split netlist: (n_res, 2) nodes and conductances."""
    r = getattr(circ, "res", None)
    if r is None:
        return np.zeros((0, 2), np.int32), np.zeros(0)
    return (np.ascontiguousarray(r, dtype=np.int32).reshape(-1, 2),
            np.ascontiguousarray(circ.res_g, dtype=np.float64))


def pattern(circ):
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    vs = np.ascontiguousarray(circ.vsrc, dtype=np.int32)
    res, _ = _resistors(circ)
    rp = np.zeros(circ.n_rows + 1, dtype=np.int32)
    cap = 16 * circ.n_dev + circ.n_rows + 4 * vs.shape[0] + 2 * res.shape[0]
    ci = np.zeros(cap, dtype=np.int32)
    nnz = C.c_int64(0)
    rc = lib().or_pattern(circ.n_nodes, circ.n_dev, _ptr(term), vs.shape[0], _ptr(vs), res.shape[0],
                          _ptr(res), _ptr(rp), _ptr(ci), C.byref(nnz))
    if rc != 0:
        raise RuntimeError(f"or_pattern failed: {rc}")
    return rp, ci[:nnz.value].copy()


def linear_stamp(circ, rp, ci, magnitude: bool = False):
    """Linear part of A (the series resistors' stamps, resistor order) and the flags
    of the entries it touches."""
    res, g = _resistors(circ)
    nnz = int(rp[-1])
    Lin = np.zeros(nnz); touched = np.zeros(nnz, np.uint8)
    rc = lib().or_linear_stamp(circ.n_nodes, res.shape[0], _ptr(res), _ptr(g), _ptr(rp), _ptr(ci), nnz,
                               _ptr(Lin), _ptr(touched), int(magnitude))
    if rc != 0:
        raise RuntimeError(f"or_linear_stamp failed: {rc}")
    return Lin, touched.astype(bool)


def stamp_map(circ, rp, ci, col, exclude: bool):
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    excl = np.ascontiguousarray(circ.exclude, dtype=np.uint8) if exclude else None
    n = circ.n_dev
    slot = np.zeros(16 * n, np.int32); sflag = np.zeros(16 * n, np.int8)
    brow = np.zeros(4 * n, np.int32); bflag = np.zeros(4 * n, np.int8)
    rc = lib().or_stamp_map(circ.n_nodes, n, _ptr(term), _ptr(excl), _ptr(col), _ptr(rp),
                            _ptr(ci), _ptr(slot), _ptr(sflag), _ptr(brow), _ptr(bflag))
    if rc != 0:
        raise RuntimeError(f"or_stamp_map failed: {rc}")
    return slot.reshape(n, 16), sflag.reshape(n, 16), brow.reshape(n, 4), bflag.reshape(n, 4)


def assemble(circ, rp, ci, nmos: dict, pmos: dict, ag0: float, hist=None, col=None,
             exclude: bool = False, x=None, W=None, L=None, VTH0=None, threads: bool = False):
    """A (CSR values) and b; col=None -> serial order, else colour replay; then the
    linear part of a split netlist's series resistors, added once per entry.
    threads=True (colour replay only): the replay spread over the OpenMP threads
    (or_assemble_omp), the same bits."""
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    pol = np.ascontiguousarray(circ.pol, dtype=np.int8)
    vs = np.ascontiguousarray(circ.vsrc, dtype=np.int32)
    vv = np.ascontiguousarray(circ.vsrc_volts, dtype=np.float64)
    excl = np.ascontiguousarray(circ.exclude, dtype=np.uint8) if (exclude and col is not None) else None
    xx = np.ascontiguousarray(circ.x if x is None else x, dtype=np.float64)
    Wa = np.ascontiguousarray(circ.W if W is None else W, dtype=np.float64)
    La = np.ascontiguousarray(circ.L if L is None else L, dtype=np.float64)
    Va = np.ascontiguousarray(circ.VTH0 if VTH0 is None else VTH0, dtype=np.float64)
    h = None if hist is None else np.ascontiguousarray(hist, dtype=np.float64)
    colp = None if col is None else np.ascontiguousarray(col, dtype=np.int32)
    res, g = _resistors(circ)
    A = np.zeros(int(rp[-1])); b = np.zeros(circ.n_rows)
    cn, cp = card(nmos), card(pmos)
    if threads and col is None:
        raise ValueError("the threaded assembly is a colour replay: give col")
    fn = lib().or_assemble_omp if threads else lib().or_assemble
    rc = fn(circ.n_nodes, circ.n_dev, _ptr(term), _ptr(pol), vs.shape[0], _ptr(vs),
                           _ptr(vv), res.shape[0], _ptr(res), _ptr(g), C.byref(cn), C.byref(cp),
                           _ptr(Wa), _ptr(La), _ptr(Va),
                           _ptr(rp), _ptr(ci), _ptr(colp), _ptr(excl), _ptr(xx), float(ag0),
                           _ptr(h), _ptr(A), _ptr(b))
    if rc != 0:
        raise RuntimeError(f"or_assemble failed: {rc}")
    return A, b


def omp_threads() -> int:
    """Threads of the OpenMP colour replay."""
    return int(lib().or_omp_threads())


def assemble_magnitude(circ, rp, ci, nmos: dict, pmos: dict, ag0: float, hist=None):
    """Per-entry sum of |device contribution| (serial)."""
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    pol = np.ascontiguousarray(circ.pol, dtype=np.int8)
    vs = np.ascontiguousarray(circ.vsrc, dtype=np.int32)
    vv = np.ascontiguousarray(circ.vsrc_volts, dtype=np.float64)
    xx = np.ascontiguousarray(circ.x, dtype=np.float64)
    h = None if hist is None else np.ascontiguousarray(hist, dtype=np.float64)
    res, g = _resistors(circ)
    A = np.zeros(int(rp[-1])); b = np.zeros(circ.n_rows)
    cn, cp = card(nmos), card(pmos)
    rc = lib().or_assemble_magnitude(circ.n_nodes, circ.n_dev, _ptr(term), _ptr(pol), vs.shape[0],
                                     _ptr(vs), _ptr(vv), res.shape[0], _ptr(res), _ptr(g), C.byref(cn),
                                     C.byref(cp), _ptr(circ.W),
                                     _ptr(circ.L), _ptr(circ.VTH0), _ptr(rp), _ptr(ci), _ptr(xx),
                                     float(ag0), _ptr(h), _ptr(A), _ptr(b))
    if rc != 0:
        raise RuntimeError(f"or_assemble_magnitude failed: {rc}")
    return np.abs(A), np.abs(b)


def hubsum(c) -> float:
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().or_hubsum(_ptr(c), c.shape[0])


def vjp(circ, rp, ci, nmos: dict, pmos: dict, ag0: float, A_bar, b_bar, hist=None,
        x=None, W=None, L=None, VTH0=None, magnitude=False):
    """Per-device gradient of <A_bar, A> + <b_bar, b> w.r.t. (W, L, VTH0); with
    magnitude=True the sum of |cotangent * sensitivity| over each device's entries,
    with magnitude="round" the device's rounding scale (or_vjp_round_scale)."""
    term = np.ascontiguousarray(circ.term, dtype=np.int32)
    pol = np.ascontiguousarray(circ.pol, dtype=np.int8)
    xx = np.ascontiguousarray(circ.x if x is None else x, dtype=np.float64)
    Wa = np.ascontiguousarray(circ.W if W is None else W, dtype=np.float64)
    La = np.ascontiguousarray(circ.L if L is None else L, dtype=np.float64)
    Va = np.ascontiguousarray(circ.VTH0 if VTH0 is None else VTH0, dtype=np.float64)
    h = None if hist is None else np.ascontiguousarray(hist, dtype=np.float64)
    Ab = np.ascontiguousarray(A_bar, dtype=np.float64)
    bb = np.ascontiguousarray(b_bar, dtype=np.float64)
    gW = np.zeros(circ.n_dev); gL = np.zeros(circ.n_dev); gV = np.zeros(circ.n_dev)
    cn, cp = card(nmos), card(pmos)
    fn = {False: lib().or_vjp, True: lib().or_vjp_magnitude, "round": lib().or_vjp_round_scale}[magnitude]
    rc = fn(circ.n_nodes, circ.n_dev, _ptr(term), _ptr(pol), C.byref(cn), C.byref(cp),
                      _ptr(Wa), _ptr(La), _ptr(Va), _ptr(rp), _ptr(ci), _ptr(xx), float(ag0),
                      _ptr(h), _ptr(Ab), _ptr(bb), _ptr(gW), _ptr(gL), _ptr(gV))
    if rc != 0:
        raise RuntimeError(f"or_vjp failed: {rc}")
    return gW, gL, gV
