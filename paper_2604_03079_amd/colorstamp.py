"""Python binding of libcolorstamp (ctypes; argument marshalling only).

Every step of the evaluate-and-stamp path runs in the HIP library; torch supplies
device memory and the current stream.  If the library is not built the import of
``lib()`` raises: there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import sys
import weakref

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_lib", "libcolorstamp.so")

VARIANTS = {"persistent": 0, "per_kernel": 1, "atomic": 2, "buffered": 3, "region": 4, "serial": 5,
            "atomic_wave": 6}
STATUS = {0: "CS_OK", -1: "CS_EINVAL", -2: "CS_ENOMEM", -3: "CS_EHIP", -4: "CS_ESTATE",
          -5: "CS_ENOTSUP", -6: "CS_EDOMAIN"}
CARD_FIELDS = ("tnom", "toxe", "ndep", "phis", "vbi", "k1", "k2", "k3", "w0", "dvt0", "dvt1",
               "dsub", "eta0", "nfactor", "cdsc", "voff", "u0", "ua", "ub", "uc", "vsat", "a0",
               "xj", "delta", "delta1", "lambda_l", "cgdo", "lint", "wint",
               "jmod", "js", "nj", "cj", "pb", "fc", "hdif", "vjmax")

# Every entry point of include/colorstamp.h.
EXPORTS = (
    "cs_circuit_create", "cs_circuit_destroy", "cs_set_resistors", "cs_build_coloring",
    "cs_build_coloring_order",
    "cs_build_stamp_map",
    "cs_get_pattern", "cs_get_stamp_map", "cs_set_models", "cs_set_params", "cs_eval_stamp",
    "cs_vjp", "cs_newton", "cs_set_newton_options", "cs_history", "cs_factor_host", "cs_set_launch", "cs_get_info", "cs_plan_regions", "cs_get_region_info",
    "cs_get_region_plan", "cs_check", "cs_set_spin_limit", "cs_set_plan_units", "cs_batch_create", "cs_batch_destroy",
    "cs_batch_layout", "cs_batch_set_params", "cs_batch_set_launch", "cs_batch_set_schedule",
    "cs_batch_get_info", "cs_batch_plan_regions", "cs_batch_get_region_info",
    "cs_batch_get_region_plan", "cs_batch_eval_stamp", "cs_batch_vjp", "cs_batch_check",
    "cs_batch_newton", "cs_batch_tune", "cs_eval_stamp_noalloc", "cs_get_region_hubs",
    "cs_batch_get_region_hubs",
    "cs_last_error",
)


class CsError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class BatchConfig(C.Structure):
    """cs_batch_config: a batched launch configuration and its measured time."""
    _fields_ = [("schedule", C.c_int32), ("block", C.c_int32), ("eval_ahead", C.c_int32),
                ("local_max_dev", C.c_int32), ("ms", C.c_double)]


class ModelCard(C.Structure):
    _fields_ = [("size", C.c_uint32)] + [(f, C.c_double) for f in CARD_FIELDS]


def make_card(d: dict) -> ModelCard:
    c = ModelCard(C.sizeof(ModelCard), *[float(d[f]) for f in CARD_FIELDS])
    return c


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libcolorstamp.so not built ({LIB_PATH}); build it with paper_2604_03079_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        i32, i64, d, p = C.c_int32, C.c_int64, C.c_double, C.c_void_p
        sig = {
            "cs_circuit_create": [i32, i32, p, p, i32, p, p, p],
            "cs_set_resistors": [p, i32, p, p],
            "cs_build_coloring": [p, p, p, p, p],
            "cs_build_coloring_order": [p, p, i32, p, p, p],
            "cs_build_stamp_map": [p, p, p],
            "cs_get_pattern": [p, p, p],
            "cs_get_stamp_map": [p, p, p, p, p],
            "cs_set_models": [p, p, p],
            "cs_set_params": [p, p, p, p, p],
            "cs_eval_stamp": [p, C.c_int, p, d, p, p, p, p],
            "cs_eval_stamp_noalloc": [p, p, d, p, p, p, p],
            "cs_vjp": [p, p, d, p, p, p, p, p, p, p],
            "cs_newton": [p, C.c_int, i32, p, d, p, i32, d, d, p, p, p, p, p, p, p],
            "cs_set_newton_options": [p, i32],
            "cs_factor_host": [p, p, p, p, p, p, p, p],
            "cs_history": [p, p, d, p, p],
            "cs_set_launch": [p, i32, i32, i32],
            "cs_get_info": [p, p, p, p, p, p, p, p, p],
            "cs_plan_regions": [p, i32],
            "cs_get_region_info": [p, p, p, p, p, p, p, p, p],
            "cs_get_region_plan": [p, p, p, p, p, p, p, p, p, p],
            "cs_get_region_hubs": [p, p, p, p],
            "cs_batch_get_region_hubs": [p, p, p, p],
            "cs_check": [p, p],
            "cs_set_spin_limit": [p, i64],
            "cs_set_plan_units": [p, i32],
            "cs_batch_create": [i32, p, p],
            "cs_batch_layout": [p, p, p, p],
            "cs_batch_set_params": [p, p, p, p, p],
            "cs_batch_set_launch": [p, i32, i32, i32],
            "cs_batch_get_info": [p, p, p, p, p, p, p, p, p],
            "cs_batch_set_schedule": [p, C.c_int],
            "cs_batch_plan_regions": [p, i32],
            "cs_batch_get_region_info": [p, p, p, p, p, p, p, p, p],
            "cs_batch_get_region_plan": [p, p, p, p, p, p, p, p, p, p],
            "cs_batch_eval_stamp": [p, p, d, p, p, p, p],
            "cs_batch_vjp": [p, p, d, p, p, p, p, p, p, p],
            "cs_batch_check": [p, p],
            "cs_batch_newton": [p, i32, p, d, p, i32, d, d, p, p, p, p, p, p, p],
            "cs_batch_tune": [p, p, p, p, p, d, p, p, i32, C.c_char_p, p, p, p, p],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.cs_circuit_destroy.argtypes = [p]
        L.cs_circuit_destroy.restype = None
        L.cs_batch_destroy.argtypes = [p]
        L.cs_batch_destroy.restype = None
        L.cs_last_error.restype = C.c_char_p
        _lib = L
    return _lib


# Handles still open.  They are destroyed by an exit hook, which runs before the
# interpreter tears its modules down and before the C runtime's exit handlers (where
# the HIP runtime and any profiler attached to it finalise): a device free issued
# from a destructor after that point would call into a runtime that is gone.
_live = weakref.WeakSet()


def _close_all():
    for o in [o for o in list(_live) if isinstance(o, Batch)] + [o for o in list(_live) if isinstance(o, Circuit)]:
        o.close()


atexit.register(_close_all)


def _check(st: int, where: str):
    if st != 0:
        raise CsError(st, where, lib().cs_last_error().decode())


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _check_layout(t, n, what):
    """Type, dtype, element count and contiguity of one device operand."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != torch.float64:
        raise TypeError(f"{what}: dtype must be torch.float64, got {t.dtype}")
    if n is not None and t.numel() != int(n):
        raise ValueError(f"{what}: expected {int(n)} elements, got {t.numel()}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")


def _check_device(t, what, device):
    if not t.is_cuda:
        raise ValueError(f"{what}: must be a CUDA tensor (the library reads and writes device memory)")
    if device is not None and t.device.index != device:
        raise ValueError(f"{what}: on cuda:{t.device.index}, the handle lives on cuda:{device}")


def _dev_ptrs(device, *specs):
    """Device addresses of caller tensors, each spec (tensor or None, element count
    or None, name), after checking what the kernels assume: contiguous torch.float64
    tensors of exactly the stated size (every operand first), then CUDA tensors on
    the handle's device.  Raises TypeError / ValueError; nothing reaches the library
    otherwise."""
    for t, n, what in specs:
        if t is not None:
            _check_layout(t, n, what)
    for t, _, what in specs:
        if t is not None:
            _check_device(t, what, device)
    return [None if t is None else C.c_void_p(t.data_ptr()) for t, _, _ in specs]


def _dev_ptr(t, n=None, what="tensor", device=None):
    """_dev_ptrs for one operand."""
    return _dev_ptrs(device, (t, n, what))[0]


def _cuda_index(t):
    """Device index of a CUDA tensor, else None (the checks then refuse it)."""
    import torch
    return t.device.index if isinstance(t, torch.Tensor) and t.is_cuda else None


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


RT_FIELDS = 12   # fields per region in the plan's region table
SOLVERS = {"levels": 0, "rocsolver": 1}
ORDERS = {"natural": 0, "largest_first": 1, "dsatur": 2}   # cs_colour_order


def _region_info(fn, h) -> dict:
    nr, mp = C.c_int32(), C.c_int32()
    ni, ns, nn, nl, nf, nfs = (C.c_int64() for _ in range(6))
    _check(fn(h, C.byref(nr), C.byref(mp), C.byref(ni), C.byref(ns), C.byref(nn), C.byref(nl),
              C.byref(nf), C.byref(nfs)), "region info")
    return dict(n_regions=nr.value, max_phases=mp.value, n_items=ni.value, n_staged=ns.value,
                n_interior=nn.value, n_links=nl.value, n_folds=nf.value, n_fold_src=nfs.value)


def _region_plan(plan_fn, info_fn, get_fn, hubs_fn, h, block, n_dev) -> dict:
    """Host planning for `block` threads per region, and a copy of the tables."""
    _check(plan_fn(h, int(block)), "plan regions")
    inf = _region_info(info_fn, h)
    t = dict(perm=np.zeros(n_dev, np.int32), phase=np.zeros(n_dev, np.uint16),
             code=np.zeros(20 * n_dev, np.int32), rtab=np.zeros(RT_FIELDS * inf["n_regions"], np.int32),
             interior=np.zeros(inf["n_interior"], np.int32), links=np.zeros(inf["n_links"], np.int32),
             item=np.zeros(4 * inf["n_items"], np.int32), fold=np.zeros(3 * inf["n_folds"], np.int32),
             fold_src=np.zeros(inf["n_fold_src"], np.int32))
    _check(get_fn(h, *[_np_ptr(t[k]) if t[k].size else None
                       for k in ("perm", "phase", "code", "rtab", "interior", "links", "item", "fold",
                                 "fold_src")]),
           "region plan")
    # hub parts: local parts, part ranges
    cnt = (C.c_int64 * 2)()
    _check(hubs_fn(h, cnt, None, None), "region hubs")
    hub = dict(hfold=np.zeros(cnt[0], np.int32), part_ptr=np.zeros(cnt[1] + 1, np.int32))
    _check(hubs_fn(h, None, _np_ptr(hub["hfold"]) if hub["hfold"].size else None, _np_ptr(hub["part_ptr"])),
           "region hubs")
    t.update(hub)
    t["code"] = t["code"].reshape(20, n_dev)
    t["rtab"] = t["rtab"].reshape(-1, RT_FIELDS)
    t["item"] = t["item"].reshape(-1, 4)
    t["fold"] = t["fold"].reshape(-1, 3)
    t.update(inf)
    return t


class Circuit:
    """One circuit behind the C-ABI.  Topology comes from numpy arrays (host)."""

    def __init__(self, n_nodes, term, pol, vsrc, vsrc_volts):
        term = np.ascontiguousarray(term, dtype=np.int32).reshape(-1, 4)
        pol = np.ascontiguousarray(pol, dtype=np.int8)
        vsrc = np.ascontiguousarray(vsrc, dtype=np.int32).reshape(-1, 2)
        vv = np.ascontiguousarray(vsrc_volts, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().cs_circuit_create(int(n_nodes), term.shape[0], _np_ptr(term), _np_ptr(pol),
                                       vsrc.shape[0], _np_ptr(vsrc), _np_ptr(vv), C.byref(h)),
               "cs_circuit_create")
        self._h = h
        _live.add(self)
        self.n_nodes = int(n_nodes)
        self.n_dev = term.shape[0]
        self.n_rows = None
        self.nnz = None
        self.n_colors = None

    @classmethod
    def from_netlist(cls, circ):
        c = cls(circ.n_nodes, circ.term, circ.pol, circ.vsrc, circ.vsrc_volts)
        if getattr(circ, "res", None) is not None and len(circ.res):
            c.set_resistors(circ.res, circ.res_g)
        return c

    def set_resistors(self, nodes, g):
        """Series resistors (linear, stamped after the FETs): (n, 2) node pairs and
        conductances in siemens.  Before build_map."""
        nodes = np.ascontiguousarray(nodes, dtype=np.int32).reshape(-1, 2)
        g = np.ascontiguousarray(g, dtype=np.float64)
        if g.shape[0] != nodes.shape[0]:
            raise ValueError("one conductance per resistor")
        _check(lib().cs_set_resistors(self._h, nodes.shape[0], _np_ptr(nodes), _np_ptr(g)),
               "cs_set_resistors")

    def close(self):
        """Destroy the library handle (device memory included); idempotent."""
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cs_circuit_destroy(h)
        self._h = None

    def __del__(self):
        # during interpreter shutdown the exit hook has already closed every handle;
        # a destructor that runs later must not call into the HIP runtime
        if not sys.is_finalizing():
            self.close()

    @property
    def handle(self):
        return self._h

    def colour(self, exclude=None, order: str = "natural"):
        """Greedy colouring; exclude = None (paper rule) or per-node flags; order =
        natural (ascending index, the paper's), largest_first or dsatur."""
        ex = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.uint8)
        col = np.zeros(self.n_dev, dtype=np.int32)
        nc = C.c_int32()
        ne = C.c_int64()
        _check(lib().cs_build_coloring_order(self._h, _np_ptr(ex), ORDERS[order], C.byref(nc), _np_ptr(col),
                                             C.byref(ne)), "cs_build_coloring_order")
        self.n_colors = nc.value
        return col, nc.value, ne.value

    def build_map(self):
        nr = C.c_int32()
        nz = C.c_int64()
        _check(lib().cs_build_stamp_map(self._h, C.byref(nr), C.byref(nz)), "cs_build_stamp_map")
        self.n_rows, self.nnz = nr.value, nz.value
        return nr.value, nz.value

    def pattern(self):
        rp = np.zeros((self.n_rows or 0) + 1, dtype=np.int32)
        ci = np.zeros(max(self.nnz or 0, 1), dtype=np.int32)
        _check(lib().cs_get_pattern(self._h, _np_ptr(rp), _np_ptr(ci)), "cs_get_pattern")
        return rp, ci[:self.nnz]

    def stamp_map(self):
        n = self.n_dev
        slot = np.zeros(16 * n, np.int32); sflag = np.zeros(16 * n, np.int8)
        brow = np.zeros(4 * n, np.int32); bflag = np.zeros(4 * n, np.int8)
        _check(lib().cs_get_stamp_map(self._h, _np_ptr(slot), _np_ptr(sflag), _np_ptr(brow),
                                      _np_ptr(bflag)), "cs_get_stamp_map")
        return slot.reshape(n, 16), sflag.reshape(n, 16), brow.reshape(n, 4), bflag.reshape(n, 4)

    def set_models(self, nmos: dict, pmos: dict):
        cn, cp = make_card(nmos), make_card(pmos)
        _check(lib().cs_set_models(self._h, C.byref(cn), C.byref(cp)), "cs_set_models")

    def set_params(self, W, L, VTH0, stream=None):
        dev = _cuda_index(W)
        n = self.n_dev
        ptrs = _dev_ptrs(dev, (W, n, "W"), (L, n, "L"), (VTH0, n, "VTH0"))
        _check(lib().cs_set_params(self._h, *ptrs, _stream(stream)), "cs_set_params")
        self._device = dev

    def set_launch(self, block: int = 0, eval_ahead: int = -1, cooperative: bool = True):
        _check(lib().cs_set_launch(self._h, int(block), int(eval_ahead), int(bool(cooperative))),
               "cs_set_launch")

    def set_spin_limit(self, spins: int):
        _check(lib().cs_set_spin_limit(self._h, int(spins)), "cs_set_spin_limit")

    def set_plan_units(self, cus: int):
        _check(lib().cs_set_plan_units(self._h, int(cus)), "cs_set_plan_units")

    def info(self) -> dict:
        nd, nr, nz = C.c_int64(), C.c_int32(), C.c_int64()
        nc, g, bl, ea, nh = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().cs_get_info(self._h, C.byref(nd), C.byref(nr), C.byref(nz), C.byref(nc),
                                 C.byref(g), C.byref(bl), C.byref(ea), C.byref(nh)), "cs_get_info")
        return dict(n_dev=nd.value, n_rows=nr.value, nnz=nz.value, n_colors=nc.value, grid=g.value,
                    block=bl.value, eval_ahead=ea.value, n_hub=nh.value)

    def region_info(self) -> dict:
        return _region_info(lib().cs_get_region_info, self._h)

    def region_plan(self, block: int = 256) -> dict:
        L = lib()
        return _region_plan(L.cs_plan_regions, L.cs_get_region_info, L.cs_get_region_plan, L.cs_get_region_hubs, self._h,
                            block, self.n_dev)

    def eval_stamp(self, x, ag0: float, hist=None, A=None, b=None, variant="persistent", stream=None):
        import torch
        if A is None:
            A = torch.empty(self.nnz, dtype=torch.float64, device=x.device)
        if b is None:
            b = torch.empty(self.n_rows, dtype=torch.float64, device=x.device)
        px, ph, pA, pb = _dev_ptrs(getattr(self, "_device", None), (x, self.n_rows, "x"),
                                   (hist, 4 * self.n_dev, "hist"), (A, self.nnz, "A"), (b, self.n_rows, "b"))
        _check(lib().cs_eval_stamp(self._h, VARIANTS[variant], px, float(ag0), ph, pA, pb, _stream(stream)),
               "cs_eval_stamp")
        return A, b

    def eval_stamp_noalloc(self, x, ag0: float, A, b, hist=None, stream=None):
        """cs_eval_stamp_noalloc: the region schedule into the caller's A and b with the
        library's per-GPU scratch array (no allocation, by this binding either)."""
        px, ph, pA, pb = _dev_ptrs(getattr(self, "_device", None), (x, self.n_rows, "x"),
                                   (hist, 4 * self.n_dev, "hist"), (A, self.nnz, "A"), (b, self.n_rows, "b"))
        _check(lib().cs_eval_stamp_noalloc(self._h, px, float(ag0), ph, pA, pb, _stream(stream)),
               "cs_eval_stamp_noalloc")
        return A, b

    def vjp(self, x, ag0: float, A_bar, b_bar, hist=None, stream=None):
        import torch
        gW = torch.empty(self.n_dev, dtype=torch.float64, device=x.device)
        gL = torch.empty_like(gW)
        gV = torch.empty_like(gW)
        n = self.n_dev
        px, ph, pa, pb, pw, pl, pv = _dev_ptrs(
            getattr(self, "_device", None), (x, self.n_rows, "x"), (hist, 4 * n, "hist"), (A_bar, self.nnz, "A_bar"),
            (b_bar, self.n_rows, "b_bar"), (gW, n, "W_bar"), (gL, n, "L_bar"), (gV, n, "VTH0_bar"))
        _check(lib().cs_vjp(self._h, px, float(ag0), ph, pa, pb, pw, pl, pv, _stream(stream)), "cs_vjp")
        return gW, gL, gV

    def check(self, stream=None):
        _check(lib().cs_check(self._h, _stream(stream)), "cs_check")

    def newton(self, x, ag0: float = 0.0, hist=None, max_iter: int = 100, vstep: float = 0.3,
               tol: float = 1e-9, variant="region", solver="levels", A=None, b=None, stream=None) -> dict:
        """Newton loop on the GPU from x (device, updated in place): iterations,
        convergence, last max |step| and the summed phase times (ms).  solver:
        "levels" (this library's kernels) or "rocsolver"."""
        import torch
        if A is None:
            A = torch.empty(self.nnz, dtype=torch.float64, device=x.device)
        if b is None:
            b = torch.empty(self.n_rows, dtype=torch.float64, device=x.device)
        it, conv, step = C.c_int32(), C.c_int32(), C.c_double()
        t = (C.c_double * 5)()
        px, ph, pA, pb = _dev_ptrs(getattr(self, "_device", None), (x, self.n_rows, "x"),
                                   (hist, 4 * self.n_dev, "hist"), (A, self.nnz, "A"), (b, self.n_rows, "b"))
        _check(lib().cs_newton(self._h, VARIANTS[variant], SOLVERS[solver], px, float(ag0), ph, int(max_iter),
                               float(vstep), float(tol), pA, pb, C.byref(it), C.byref(conv),
                               C.byref(step), t, _stream(stream)), "cs_newton")
        return dict(iterations=it.value, converged=bool(conv.value), last_step=step.value,
                    ms=dict(stamp=t[0], refactor=t[1], solve=t[2], update=t[3], host_factor=t[4]))

    def set_newton_options(self, programmed_rows: bool = True, upper_runs: bool = True):
        """Launch schedule of the level-scheduled solver (same bits either way)."""
        flags = (0 if programmed_rows else 1) | (0 if upper_runs else 2)
        _check(lib().cs_set_newton_options(self._h, flags), "cs_set_newton_options")

    def history(self, x, ag0: float, out=None, stream=None):
        """ag0 * terminal charges of every device at x: the history terms (n_dev, 4)
        of the next backward-Euler step."""
        import torch
        if out is None:
            out = torch.empty((self.n_dev, 4), dtype=torch.float64, device=x.device)
        px, po = _dev_ptrs(getattr(self, "_device", None), (x, self.n_rows, "x"), (out, 4 * self.n_dev, "hist_out"))
        _check(lib().cs_history(self._h, px, float(ag0), po, _stream(stream)), "cs_history")
        return out

    def transient(self, x, h: float, n_steps: int, nodes=None, **newton_kw):
        """Backward-Euler transient from x (device, updated in place): per step the
        history terms at the present point, then the Newton loop with ag0 = 1/h.
        Returns the node voltages (rows of `nodes`, default all) after every step
        (n_steps + 1 rows, the start first) and the Newton iteration counts."""
        import torch
        ag0 = 1.0 / h
        rows = torch.arange(self.n_rows, device=x.device) if nodes is None else \
            torch.as_tensor(np.asarray(nodes) - 1, device=x.device)
        wave = [x[rows].clone()]
        iters = []
        hist = torch.empty((self.n_dev, 4), dtype=torch.float64, device=x.device)
        for _ in range(n_steps):
            self.history(x, ag0, hist)
            r = self.newton(x, ag0, hist, **newton_kw)
            if not r["converged"]:
                raise CsError(-6, "transient", f"Newton did not converge at step {len(iters) + 1}")
            iters.append(r["iterations"])
            wave.append(x[rows].clone())
        return torch.stack(wave), iters

    def factor_host(self, A_host):
        """The host LU the Newton loop starts from: P, Q and T = (L - I) + U (CSR)."""
        Ah = np.ascontiguousarray(A_host, dtype=np.float64)
        nz = C.c_int64()
        L = lib()
        _check(L.cs_factor_host(self._h, _np_ptr(Ah), C.byref(nz), None, None, None, None, None), "cs_factor_host")
        n = self.n_rows
        P, Q = np.zeros(n, np.int32), np.zeros(n, np.int32)
        Tp, Ti, Tx = np.zeros(n + 1, np.int32), np.zeros(max(nz.value, 1), np.int32), np.zeros(max(nz.value, 1))
        _check(L.cs_factor_host(self._h, _np_ptr(Ah), C.byref(nz), _np_ptr(P), _np_ptr(Q), _np_ptr(Tp), _np_ptr(Ti),
                                _np_ptr(Tx)), "cs_factor_host")
        return P, Q, Tp, Ti[:nz.value], Tx[:nz.value]


def prepare(circ, exclude: bool = True, nmos=None, pmos=None, order: str = "natural"):
    """Circuit from a generator netlist: coloured (rails excluded or not, in the given
    vertex order) and mapped."""
    from . import netgen
    c = Circuit.from_netlist(circ)
    c.colour(circ.exclude if exclude else None, order)
    c.build_map()
    c.set_models(nmos or netgen.default_card(1), pmos or netgen.default_card(-1))
    return c


class Batch:
    """Many prepared circuits stamped in one launch (packed layouts, see cs_batch_layout)."""

    def __init__(self, circuits):
        self.circuits = list(circuits)
        n = len(self.circuits)
        arr = (C.c_void_p * n)(*[c.handle for c in self.circuits])
        h = C.c_void_p()
        _check(lib().cs_batch_create(n, arr, C.byref(h)), "cs_batch_create")
        self._h = h
        _live.add(self)
        self.dev_off = np.zeros(n + 1, np.int64)
        self.row_off = np.zeros(n + 1, np.int64)
        self.nnz_off = np.zeros(n + 1, np.int64)
        _check(lib().cs_batch_layout(h, _np_ptr(self.dev_off), _np_ptr(self.row_off),
                                     _np_ptr(self.nnz_off)), "cs_batch_layout")
        self.n_dev = int(self.dev_off[-1])
        self.n_rows = int(self.row_off[-1])
        self.nnz = int(self.nnz_off[-1])

    def close(self):
        """Destroy the batch handle (its circuits stay open); idempotent."""
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.cs_batch_destroy(h)
        self._h = None

    def __del__(self):
        if not sys.is_finalizing():
            self.close()

    def set_launch(self, block: int = 0, eval_ahead: int = -1, local_max_dev: int = 0,
                   schedule: str = "persistent"):
        _check(lib().cs_batch_set_launch(self._h, int(block), int(eval_ahead), int(local_max_dev)),
               "cs_batch_set_launch")
        _check(lib().cs_batch_set_schedule(self._h, VARIANTS[schedule]), "cs_batch_set_schedule")

    def region_info(self) -> dict:
        return _region_info(lib().cs_batch_get_region_info, self._h)

    def region_plan(self, block: int = 256) -> dict:
        L = lib()
        return _region_plan(L.cs_batch_plan_regions, L.cs_batch_get_region_info,
                            L.cs_batch_get_region_plan, L.cs_batch_get_region_hubs, self._h, block, self.n_dev)

    def set_params(self, W, L, VTH0, stream=None):
        dev = _cuda_index(W)
        n = self.n_dev
        ptrs = _dev_ptrs(dev, (W, n, "W"), (L, n, "L"), (VTH0, n, "VTH0"))
        _check(lib().cs_batch_set_params(self._h, *ptrs, _stream(stream)), "cs_batch_set_params")
        self._device = dev

    def info(self) -> dict:
        nd, nr, nz = C.c_int64(), C.c_int64(), C.c_int64()
        mc, g, bl, ea, nl = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().cs_batch_get_info(self._h, C.byref(nd), C.byref(nr), C.byref(nz), C.byref(mc),
                                       C.byref(g), C.byref(bl), C.byref(ea), C.byref(nl)),
               "cs_batch_get_info")
        return dict(n_dev=nd.value, n_rows=nr.value, nnz=nz.value, max_colors=mc.value, grid=g.value,
                    block=bl.value, eval_ahead=ea.value, n_local=nl.value)

    def eval_stamp(self, x, ag0: float, hist=None, A=None, b=None, stream=None):
        import torch
        if A is None:
            A = torch.empty(self.nnz, dtype=torch.float64, device=x.device)
        if b is None:
            b = torch.empty(self.n_rows, dtype=torch.float64, device=x.device)
        px, ph, pA, pb = _dev_ptrs(getattr(self, "_device", None), (x, self.n_rows, "x"),
                                   (hist, 4 * self.n_dev, "hist"), (A, self.nnz, "A"), (b, self.n_rows, "b"))
        _check(lib().cs_batch_eval_stamp(self._h, px, float(ag0), ph, pA, pb, _stream(stream)), "cs_batch_eval_stamp")
        return A, b

    def vjp(self, x, ag0: float, A_bar, b_bar, hist=None, stream=None):
        import torch
        gW = torch.empty(self.n_dev, dtype=torch.float64, device=x.device)
        gL = torch.empty_like(gW)
        gV = torch.empty_like(gW)
        n = self.n_dev
        px, ph, pa, pb, pw, pl, pv = _dev_ptrs(
            getattr(self, "_device", None), (x, self.n_rows, "x"), (hist, 4 * n, "hist"), (A_bar, self.nnz, "A_bar"),
            (b_bar, self.n_rows, "b_bar"), (gW, n, "W_bar"), (gL, n, "L_bar"), (gV, n, "VTH0_bar"))
        _check(lib().cs_batch_vjp(self._h, px, float(ag0), ph, pa, pb, pw, pl, pv, _stream(stream)), "cs_batch_vjp")
        return gW, gL, gV

    def check(self, stream=None):
        _check(lib().cs_batch_check(self._h, _stream(stream)), "cs_batch_check")

    def tune(self, W, L, VTH0, x, ag0: float, A, b, reps: int = 8, cache_path: str | None = None,
             stream=None) -> dict:
        """cs_batch_tune: time every candidate launch configuration (graph replays)
        and apply the fastest; returns it with its time, the number of candidates
        timed and whether it came from the cache file."""
        dev = _cuda_index(W)
        n = self.n_dev
        cfg, tried, cached = BatchConfig(), C.c_int32(), C.c_int32()
        pw, pl, pv, px, pA, pb = _dev_ptrs(dev, (W, n, "W"), (L, n, "L"), (VTH0, n, "VTH0"), (x, self.n_rows, "x"),
                                           (A, self.nnz, "A"), (b, self.n_rows, "b"))
        _check(lib().cs_batch_tune(self._h, pw, pl, pv, px, float(ag0), pA, pb, int(reps),
                                   None if cache_path is None else os.fsencode(cache_path), C.byref(cfg),
                                   C.byref(tried), C.byref(cached), _stream(stream)), "cs_batch_tune")
        self._device = dev
        sched = {v: k for k, v in VARIANTS.items()}[cfg.schedule]
        return dict(schedule=sched, block=cfg.block, eval_ahead=cfg.eval_ahead, local_max_dev=cfg.local_max_dev,
                    ms=cfg.ms, tried=tried.value, cached=bool(cached.value))

    def newton(self, x, ag0: float = 0.0, hist=None, max_iter: int = 100, vstep: float = 0.3,
               tol: float = 1e-9, solver="levels", A=None, b=None, stream=None) -> dict:
        """Newton loop over every circuit at once from the packed x (device, updated
        in place); returns as Circuit.newton."""
        import torch
        if A is None:
            A = torch.empty(self.nnz, dtype=torch.float64, device=x.device)
        if b is None:
            b = torch.empty(self.n_rows, dtype=torch.float64, device=x.device)
        it, conv, step = C.c_int32(), C.c_int32(), C.c_double()
        t = (C.c_double * 5)()
        px, ph, pA, pb = _dev_ptrs(getattr(self, "_device", None), (x, self.n_rows, "x"),
                                   (hist, 4 * self.n_dev, "hist"), (A, self.nnz, "A"), (b, self.n_rows, "b"))
        _check(lib().cs_batch_newton(self._h, SOLVERS[solver], px, float(ag0), ph, int(max_iter), float(vstep),
                                     float(tol), pA, pb,
                                     C.byref(it), C.byref(conv), C.byref(step), t, _stream(stream)),
               "cs_batch_newton")
        return dict(iterations=it.value, converged=bool(conv.value), last_step=step.value,
                    ms=dict(stamp=t[0], refactor=t[1], solve=t[2], update=t[3], host_factor=t[4]))

    def history(self, x, ag0: float, out=None, stream=None):
        """Packed history terms (n_dev, 4) of the next backward-Euler step: each
        circuit's cs_history on its slice of the packed x, with the member
        circuits' own parameters (per_circuit_params gives them the batch's)."""
        import torch
        if out is None:
            out = torch.empty((self.n_dev, 4), dtype=torch.float64, device=x.device)
        for i, c in enumerate(self.circuits):
            r0, r1 = int(self.row_off[i]), int(self.row_off[i + 1])
            a, z = int(self.dev_off[i]), int(self.dev_off[i + 1])
            c.history(x[r0:r1], ag0, out[a:z], stream)
        return out

    def transient(self, x, h: float, n_steps: int, **newton_kw):
        """Backward-Euler transient of every circuit at once from the packed x
        (device, updated in place), as Circuit.transient: the packed rows after every
        step (n_steps + 1 rows, the start first) and the Newton iteration counts.
        The history terms use the member circuits' parameters (per_circuit_params)."""
        import torch
        ag0 = 1.0 / h
        wave = [x.clone()]
        iters = []
        hist = torch.empty((self.n_dev, 4), dtype=torch.float64, device=x.device)
        for _ in range(n_steps):
            self.history(x, ag0, hist)
            r = self.newton(x, ag0, hist, **newton_kw)
            if not r["converged"]:
                raise CsError(-6, "transient", f"Newton did not converge at step {len(iters) + 1}")
            iters.append(r["iterations"])
            wave.append(x.clone())
        return torch.stack(wave), iters

    def per_circuit_params(self, W, L, VTH0):
        """Give every member circuit its slice of the packed parameters."""
        for i, c in enumerate(self.circuits):
            a, z = int(self.dev_off[i]), int(self.dev_off[i + 1])
            c.set_params(W[a:z], L[a:z], VTH0[a:z])

    def per_circuit_eval(self, x, ag0, A, b, variant="persistent"):
        """The comparison schedule: one launch per circuit on packed slices."""
        for i, c in enumerate(self.circuits):
            r0, r1 = int(self.row_off[i]), int(self.row_off[i + 1])
            z0, z1 = int(self.nnz_off[i]), int(self.nnz_off[i + 1])
            c.eval_stamp(x[r0:r1], ag0, None, A[z0:z1], b[r0:r1], variant)
        return A, b


def _torch_function():
    import torch

    class StampFn(torch.autograd.Function):
        """(W, L, VTH0, x) -> (A, b) with the hand-written adjoint in backward.

        The gradient with respect to x is not provided (None)."""

        @staticmethod
        def forward(ctx, circuit, W, L, VTH0, x, ag0, variant):
            circuit.set_params(W, L, VTH0)
            A, b = circuit.eval_stamp(x, ag0, variant=variant)
            ctx.save_for_backward(W, L, VTH0, x)
            ctx.circuit = circuit
            ctx.ag0 = ag0
            return A, b

        @staticmethod
        def backward(ctx, A_bar, b_bar):
            W, L, VTH0, x = ctx.saved_tensors
            c = ctx.circuit
            if A_bar is None:
                A_bar = torch.zeros(c.nnz, dtype=torch.float64, device=x.device)
            if b_bar is None:
                b_bar = torch.zeros(c.n_rows, dtype=torch.float64, device=x.device)
            c.set_params(W, L, VTH0)
            gW, gL, gV = c.vjp(x, ctx.ag0, A_bar.contiguous(), b_bar.contiguous())
            return None, gW, gL, gV, None, None, None

    return StampFn


_STAMPFN = None


def stamp(circuit, W, L, VTH0, x, ag0: float = 1e12, variant: str = "persistent"):
    """Differentiable evaluate-and-stamp: returns (A_val, b); backward gives dW, dL, dVTH0."""
    global _STAMPFN
    if _STAMPFN is None:
        _STAMPFN = _torch_function()
    return _STAMPFN.apply(circuit, W, L, VTH0, x, ag0, variant)
