"""Binding of the general-geometry knitting calls declared in ``include/knit_graph.h``.

Argument marshalling only: the plan is built by the library's host code and
every arithmetic step runs in the HIP kernel of ``libknit.so``.  A system is
given as a CSR hopping graph (``row_ptr``, ``col``) with one norb x norb block
per directed edge, on-site blocks per site, and leads as lists of sites.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import knit as K

_lib = K._lib
c_i32, c_i64, c_dbl, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t

KNIT_GRAPH_MAX_LEADS = 16
KNIT_GRAPH_MAX_PAIRS = 16
KNIT_GRAPH_MAX_DIM = 2048


class KnitGraphLead(ctypes.Structure):
    _fields_ = [("nsite", c_i32), ("reserved", c_i32), ("sites", c_vp)]


class KnitGraphInfo(ctypes.Structure):
    _fields_ = [("nsite", c_i32), ("norb", c_i32), ("n_leads", c_i32), ("max_slots", c_i32), ("dim", c_i32),
                ("lead_dim", c_i32), ("max_pairs", c_i32), ("n_steps", c_i32), ("sigma_size", c_i64),
                ("nnz", c_i64), ("update_flops", c_dbl), ("update_bytes", c_dbl), ("block", c_i32),
                ("reserved", c_i32)]


assert ctypes.sizeof(KnitGraphLead) == 16
assert ctypes.sizeof(KnitGraphInfo) == 72

GRAPH_PROBLEM_DTYPE = np.dtype([("E", "<f8"), ("onsite_off", "<i8"), ("sigma_off", "<i8"), ("gll_off", "<i8")])
assert GRAPH_PROBLEM_DTYPE.itemsize == 32

_lib.knit_graph_plan_create.restype = c_i32
_lib.knit_graph_plan_create.argtypes = [c_i32, c_i32, c_vp, c_vp, c_i32, ctypes.POINTER(KnitGraphLead), c_vp,
                                        ctypes.POINTER(c_vp)]
_lib.knit_graph_plan_create_blocked.restype = c_i32
_lib.knit_graph_plan_create_blocked.argtypes = [c_i32, c_i32, c_vp, c_vp, c_i32, ctypes.POINTER(KnitGraphLead), c_vp,
                                                c_i32, ctypes.POINTER(c_vp)]
_lib.knit_graph_plan_info.restype = c_i32
_lib.knit_graph_plan_info.argtypes = [c_vp, ctypes.POINTER(KnitGraphInfo)]
_lib.knit_graph_plan_order.restype = c_i32
_lib.knit_graph_plan_order.argtypes = [c_vp, c_vp]
_lib.knit_graph_plan_destroy.restype = None
_lib.knit_graph_plan_destroy.argtypes = [c_vp]
_lib.knit_graph_workspace.restype = c_sz
_lib.knit_graph_workspace.argtypes = [c_vp, c_i32]
_lib.knit_graph_transmission.restype = c_i32
_lib.knit_graph_transmission.argtypes = [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]

EXPORTED = ["knit_graph_plan_create", "knit_graph_plan_create_blocked", "knit_graph_plan_info", "knit_graph_plan_order", "knit_graph_plan_destroy",
            "knit_graph_workspace", "knit_graph_transmission"]


class GraphPlan:
    """Owns a knit_graph_plan handle (destroyed with the object)."""

    _destroy = _lib.knit_graph_plan_destroy

    def __init__(self, nsite: int, norb: int, row_ptr, col, leads, order=None, block: int | None = None):
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.leads = [np.ascontiguousarray(l, dtype=np.int32) for l in leads]
        arr = (KnitGraphLead * max(1, len(self.leads)))()
        for k, l in enumerate(self.leads):
            arr[k] = KnitGraphLead(len(l), 0, l.ctypes.data)
        ordp = None
        if order is not None:
            self._order_in = np.ascontiguousarray(order, dtype=np.int32)
            ordp = self._order_in.ctypes.data
        h = c_vp()
        self.handle = None
        colp = self.col.ctypes.data if len(self.col) else None
        if block is None:   # site by site
            code = _lib.knit_graph_plan_create(int(nsite), int(norb), self.row_ptr.ctypes.data, colp,
                                               len(self.leads), arr, ordp, ctypes.byref(h))
        else:               # `block` sites per step (0: automatic)
            code = _lib.knit_graph_plan_create_blocked(int(nsite), int(norb), self.row_ptr.ctypes.data, colp,
                                                       len(self.leads), arr, ordp, int(block), ctypes.byref(h))
        self.code = code
        if code == K.KNIT_OK:
            self.handle = h.value

    def ok(self) -> bool:
        return self.handle is not None

    def info(self) -> dict:
        inf = KnitGraphInfo()
        K._check(_lib.knit_graph_plan_info(self.handle, ctypes.byref(inf)), "knit_graph_plan_info")
        return {f: getattr(inf, f) for f, _ in KnitGraphInfo._fields_}

    def order(self) -> np.ndarray:
        n = self.info()["nsite"]
        out = np.zeros(n, dtype=np.int32)
        K._check(_lib.knit_graph_plan_order(self.handle, out.ctypes.data), "knit_graph_plan_order")
        return out

    def workspace(self, P: int) -> int:
        return int(_lib.knit_graph_workspace(self.handle, int(P)))

    def __del__(self):
        if getattr(self, "handle", None):
            self._destroy(self.handle)
            self.handle = None


def plan_create(nsite, norb, row_ptr, col, leads, order=None, block=None) -> GraphPlan:
    p = GraphPlan(nsite, norb, row_ptr, col, leads, order, block)
    K._check(p.code, "knit_graph_plan_create" if block is None else "knit_graph_plan_create_blocked")
    return p


def knit_graph_transmission(plan: GraphPlan, probs: torch.Tensor, P: int, hop: torch.Tensor, onsite: torch.Tensor,
                            sigma: torch.Tensor, want_gll: bool = False, gll_size: int | None = None,
                            ws: torch.Tensor | None = None, stream=None):
    """T [P, K, K] (float64) and, if want_gll, the lead-site block of G (complex128, as laid out by
    the problems' gll_off; gll_size elements).  probs: uint8 device tensor of GRAPH_PROBLEM_DTYPE rows."""
    inf = plan.info()
    dev = hop.device if hop is not None and hop.numel() else onsite.device
    Kl = inf["n_leads"]
    T = torch.empty((P, Kl, Kl), dtype=torch.float64, device=dev)
    st = torch.empty(P, dtype=torch.int32, device=dev)
    GLL = None
    if want_gll:
        GLL = torch.empty(gll_size if gll_size is not None else P * inf["lead_dim"] ** 2, dtype=torch.complex128,
                          device=dev)
    need = plan.workspace(P)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    code = _lib.knit_graph_transmission(plan.handle, K._ptr(probs), int(P), K._ptr(hop), K._ptr(onsite),
                                        K._ptr(sigma), K._ptr(T), K._ptr(GLL), K._ptr(st), K._ptr(ws), ws.numel(),
                                        K._stream(stream))
    K._check(code, "knit_graph_transmission")
    return T, GLL, st


def problem_table(E, onsite_off, sigma_off, gll_off=None) -> np.ndarray:
    E = np.atleast_1d(np.asarray(E, dtype=np.float64))
    t = np.zeros(len(E), dtype=GRAPH_PROBLEM_DTYPE)
    t["E"] = E
    t["onsite_off"] = onsite_off
    t["sigma_off"] = sigma_off
    t["gll_off"] = 0 if gll_off is None else gll_off
    return t
