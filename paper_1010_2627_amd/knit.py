"""Python binding of libknit (ctypes): argument marshalling only.

Every function here forwards to the C entry point of the same name declared
in ``include/knit.h``; all arithmetic of the transport path runs in the HIP
kernels of ``libknit.so``.  PyTorch provides device memory and the stream.
If the library is not built this module raises at import time: there is no
fallback path.
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libknit.so")

KNIT_OK, KNIT_E_ARG, KNIT_E_DEVICE, KNIT_E_WORKSPACE, KNIT_E_UNSUPPORTED, KNIT_E_SCRATCH = 0, -1, -2, -3, -4, -5
KNIT_NOALLOC_SCRATCH_BYTES = 128 << 20
KNIT_NOALLOC_MAX_PROBLEMS = 1048576
KNIT_P_OK, KNIT_P_SINGULAR, KNIT_P_NOCONV, KNIT_P_NONFINITE, KNIT_P_FALLBACK = 0, 1, 2, 4, 8
KNIT_FP64, KNIT_FP32_REFINE, KNIT_FP32 = 0, 1, 2
PRECISIONS = {"fp64": KNIT_FP64, "fp32_refine": KNIT_FP32_REFINE, "fp32": KNIT_FP32}
KNIT_MAX_STRIPS = 64

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1010_2627_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

c_i32, c_i64, c_dbl, c_vp, c_sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t


class KnitStrip(ctypes.Structure):
    _fields_ = [("M", c_i32), ("norb", c_i32), ("H0", c_vp), ("vcol", c_vp), ("vblk", c_vp), ("V", c_vp),
                ("onsite_dense", c_i32), ("h0_band", c_i32)]


assert ctypes.sizeof(KnitStrip) == 48


PROBLEM_DTYPE = np.dtype([("strip", "<i4"), ("L", "<i4"), ("E", "<f8"), ("onsite_off", "<i8"),
                          ("sigma_off", "<i8"), ("out_off", "<i8"), ("ldos_off", "<i8")], align=True)
assert PROBLEM_DTYPE.itemsize == 48

_SP = ctypes.POINTER(KnitStrip)

_lib.knit_abi_version.restype = c_i32
_lib.knit_status_string.restype = ctypes.c_char_p
_lib.knit_status_string.argtypes = [c_i32]
_lib.knit_lead_selfenergy_workspace.restype = c_sz
_lib.knit_lead_selfenergy_workspace.argtypes = [_SP, c_i32]
_lib.knit_lead_selfenergy.restype = c_i32
_lib.knit_lead_selfenergy.argtypes = [_SP, c_i32, c_vp, c_i32, c_dbl, c_dbl, c_i32, c_vp, c_vp, c_vp,
                                      c_vp, c_sz, c_vp]
_lib.knit_rgf_sweep_workspace.restype = c_sz
_lib.knit_rgf_sweep_workspace.argtypes = [_SP, c_i32, c_vp, c_i32, c_i32, c_i32]
_lib.knit_rgf_sweep.restype = c_i32
_lib.knit_rgf_sweep.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp,
                                c_vp, c_vp, c_vp, c_sz, c_vp]
_lib.knit_rgf_sweep_noalloc.restype = c_i32
_lib.knit_rgf_sweep_noalloc.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp,
                                        c_vp, c_vp, c_vp]
_lib.knit_transmission.restype = c_i32
_lib.knit_transmission.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp,
                                   c_vp, c_vp, c_vp]
_lib.knit_ldos_workspace.restype = c_sz
_lib.knit_ldos_workspace.argtypes = [_SP, c_i32, c_vp, c_i32, c_i32, c_i32]
_lib.knit_ldos.restype = c_i32
_lib.knit_ldos.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_i32, c_i32, c_vp, c_vp,
                           c_vp, c_sz, c_vp]

_lib.knit_gamma_factor.restype = c_i32
_lib.knit_gamma_factor.argtypes = [c_i32, c_vp, c_i32, c_dbl, c_vp, c_vp, c_vp]
_lib.knit_rgf_sweep_projected.restype = c_i32
_lib.knit_rgf_sweep_projected.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp,
                                          c_vp, c_vp, c_vp, c_sz, c_vp]
_lib.knit_transmission_eigenvalues_workspace.restype = c_sz
_lib.knit_transmission_eigenvalues_workspace.argtypes = [_SP, c_i32, c_vp, c_i32]
_lib.knit_transmission_eigenvalues.restype = c_i32
_lib.knit_transmission_eigenvalues.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp,
                                               c_vp, c_vp, c_sz, c_vp]
_lib.knit_local_observables_workspace.restype = c_sz
_lib.knit_local_observables_workspace.argtypes = [_SP, c_i32, c_vp, c_i32, c_i32]
_lib.knit_local_observables.restype = c_i32
_lib.knit_local_observables.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp, c_vp,
                                        c_vp, c_vp, c_vp, c_vp, c_sz, c_vp]
_lib.knit_conductance_matrix_workspace.restype = c_sz
_lib.knit_conductance_matrix_workspace.argtypes = [_SP, c_i32, c_vp, c_i32, c_i32, c_i32]
_lib.knit_conductance_matrix.restype = c_i32
_lib.knit_conductance_matrix.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_vp,
                                         c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_sz, c_vp]
_lib.knit_transmission_projected.restype = c_i32
_lib.knit_transmission_projected.argtypes = [_SP, c_i32, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]


class KnitSweepTuning(ctypes.Structure):
    _fields_ = [("threads", c_i32), ("wg_per_cu", c_i32), ("order", c_i32), ("outer", c_i32)]


KNIT_TUNING_CLASSES = 16
_lib.knit_sweep_tuning_set.restype = c_i32
_lib.knit_sweep_tuning_set.argtypes = [c_i32, c_i32, ctypes.POINTER(KnitSweepTuning)]
_lib.knit_sweep_tuning_get.restype = c_i32
_lib.knit_sweep_tuning_get.argtypes = [c_i32, c_i32, ctypes.POINTER(KnitSweepTuning)]

_lib.knit_set_selfenergy_products.restype = c_i32
_lib.knit_set_selfenergy_products.argtypes = [c_i32]
_lib.knit_get_selfenergy_products.restype = c_i32
_lib.knit_get_selfenergy_products.argtypes = []
KNIT_PRODUCTS_VECTOR, KNIT_PRODUCTS_INT8 = 0, 1

_lib.knit_set_refine_threshold.restype = c_i32
_lib.knit_set_refine_threshold.argtypes = [c_dbl]
_lib.knit_get_refine_threshold.restype = c_dbl
_lib.knit_get_refine_threshold.argtypes = []

EXPORTED = ["knit_set_selfenergy_products", "knit_get_selfenergy_products",
            "knit_set_refine_threshold", "knit_get_refine_threshold", "knit_abi_version", "knit_status_string", "knit_lead_selfenergy_workspace",
            "knit_lead_selfenergy", "knit_rgf_sweep_workspace", "knit_rgf_sweep",
            "knit_transmission", "knit_ldos_workspace", "knit_ldos", "knit_sweep_tuning_set",
            "knit_sweep_tuning_get", "knit_gamma_factor", "knit_rgf_sweep_projected",
            "knit_transmission_projected", "knit_rgf_sweep_noalloc", "knit_transmission_eigenvalues_workspace",
            "knit_transmission_eigenvalues", "knit_local_observables_workspace", "knit_local_observables",
            "knit_conductance_matrix_workspace", "knit_conductance_matrix"]


class KnitError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code


def abi_version() -> int:
    return int(_lib.knit_abi_version())


def status_string(code: int) -> str:
    return _lib.knit_status_string(int(code)).decode()


def tuning_class(Mp: int) -> int:
    """Padded-slice class of the tuning table: Mp = 32 * ceil(M / 32), class Mp / 32 - 1."""
    return (int(Mp) + 31) // 32 - 1


def knit_sweep_tuning_set(precision, cls: int, threads: int | None = None, wg_per_cu: int = 1,
                          order: int = 1, outer: int = 64):
    """Set (or, with threads=None, reset to the default) one entry of the sweep tuning table."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    t = None if threads is None else ctypes.byref(KnitSweepTuning(int(threads), int(wg_per_cu), int(order),
                                                                   int(outer)))
    _check(_lib.knit_sweep_tuning_set(prec, int(cls), t), "knit_sweep_tuning_set")


def knit_set_refine_threshold(threshold: float):
    """Largest ||I - A_n X0||_F (first residual of a slice's FP32 inverse) the refinement may
    start from before the problem is recomputed in FP64 (KNIT_P_FALLBACK)."""
    _check(_lib.knit_set_refine_threshold(float(threshold)), "knit_set_refine_threshold")


def knit_set_selfenergy_products(mode: int):
    """KNIT_PRODUCTS_INT8 (digit planes on the INT8 matrix cores) or KNIT_PRODUCTS_VECTOR."""
    _check(_lib.knit_set_selfenergy_products(int(mode)), "knit_set_selfenergy_products")


def knit_get_selfenergy_products() -> int:
    return int(_lib.knit_get_selfenergy_products())


def knit_get_refine_threshold() -> float:
    return float(_lib.knit_get_refine_threshold())


def knit_sweep_tuning_get(precision, cls: int) -> dict:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    t = KnitSweepTuning()
    _check(_lib.knit_sweep_tuning_get(prec, int(cls), ctypes.byref(t)), "knit_sweep_tuning_get")
    return {"threads": t.threads, "wg_per_cu": t.wg_per_cu, "order": t.order, "outer": t.outer}


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, torch.Tensor):
        return t.data_ptr() if t.numel() > 0 else None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return int(t)


def _stream(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check(code: int, where: str):
    if code != KNIT_OK:
        raise KnitError(code, where)


def _z(t: torch.Tensor) -> torch.Tensor:
    assert t.dtype == torch.complex128 and t.is_contiguous()
    return t


# ---------------------------------------------------------------- device-side inputs

@dataclass
class DeviceStrip:
    """A strip class resident on the GPU (tensors keep the memory alive)."""

    M: int
    norb: int
    H0: torch.Tensor             # [M, M] complex128
    vcol: torch.Tensor | None    # [W] int32 (block-monomial V)
    vblk: torch.Tensor | None    # [W, norb, norb] complex128 (block-monomial V)
    V: torch.Tensor | None = None   # [M, M] complex128 (dense V)
    onsite_dense: bool = False
    h0_band: int = 0             # site-block half-bandwidth of H0 (0: read all of it)

    @classmethod
    def from_host(cls, strip, device="cuda"):
        dense = getattr(strip, "V", None) is not None
        t = lambda a, dt=None: torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(device)
        return cls(strip.M, strip.norb, t(strip.H0),
                   None if dense else t(strip.vcol, np.int32),
                   None if dense else t(strip.vblk),
                   t(strip.V) if dense else None,
                   bool(getattr(strip, "onsite_dense", False)), h0_band_of(strip.H0, strip.norb))

    def c(self) -> KnitStrip:
        return KnitStrip(self.M, self.norb, _ptr(self.H0), _ptr(self.vcol), _ptr(self.vblk), _ptr(self.V),
                         int(self.onsite_dense), int(self.h0_band))


def h0_band_of(H0, norb: int) -> int:
    """Largest |a - c| over the nonzero site blocks (a, c) of a host H0, or 0 (read all of H0)
    when that spans the slice anyway."""
    W = H0.shape[0] // norb
    nz = np.abs(np.asarray(H0).reshape(W, norb, W, norb)).max(axis=(1, 3)) != 0
    a, c = np.nonzero(nz)
    b = int(np.abs(a - c).max()) if len(a) else 0
    return b if 0 < b < W - 1 else 0


def strip_table(strips) -> ctypes.Array:
    arr = (KnitStrip * len(strips))()
    for i, s in enumerate(strips):
        arr[i] = s.c() if isinstance(s, DeviceStrip) else s
    return arr


@dataclass
class ProblemTable:
    host: np.ndarray          # PROBLEM_DTYPE [P]
    dev: torch.Tensor         # uint8 [P * 48] on the device

    @classmethod
    def from_host(cls, host: np.ndarray, device="cuda"):
        host = np.ascontiguousarray(host, dtype=PROBLEM_DTYPE)
        dev = torch.from_numpy(host.view(np.uint8).copy()).to(device)
        return cls(host, dev)

    @property
    def P(self) -> int:
        return int(self.host.shape[0])


# ---------------------------------------------------------------- entry points

def knit_lead_selfenergy(strip: DeviceStrip, side: int, E: torch.Tensor, eta: float = 1e-16,
                         tol: float = 1e-16, max_iter: int = 100, stream=None):
    """Sigma of the left (side 0) or right (side 1) lead, or of both (side 2), at energies E
    (device float64 [nE]).

    Returns (sigma, iters [nE] int32, status [nE] int32), all on the device; sigma is
    [nE, M, M] complex128, or [2, nE, M, M] (left, right) for side 2.
    """
    assert E.dtype == torch.float64 and E.is_cuda and E.is_contiguous()
    nE = E.numel()
    dev = E.device
    shape = (2, nE, strip.M, strip.M) if side == 2 else (nE, strip.M, strip.M)
    sigma = torch.empty(shape, dtype=torch.complex128, device=dev)
    iters = torch.zeros(nE, dtype=torch.int32, device=dev)
    status = torch.zeros(nE, dtype=torch.int32, device=dev)
    cs = strip.c()
    wsz = _lib.knit_lead_selfenergy_workspace(ctypes.byref(cs), nE)
    ws = torch.empty(max(int(wsz), 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_lead_selfenergy(ctypes.byref(cs), int(side), _ptr(E), nE, float(eta), float(tol),
                                     int(max_iter), _ptr(sigma), _ptr(iters), _ptr(status), _ptr(ws),
                                     wsz, _stream(stream))
    _check(code, "knit_lead_selfenergy")
    return sigma, iters, status


def knit_rgf_sweep(strips, probs: ProblemTable, onsite: torch.Tensor, sigmaL: torch.Tensor,
                   sigmaR: torch.Tensor, precision="fp64", G1N: torch.Tensor = None,
                   GN1: torch.Tensor | bool = False, GNN: torch.Tensor | bool = False, stream=None,
                   workspace: torch.Tensor | None = None):
    """Slice sweep for every problem of ``probs``; returns (G1N, GN1|None, GNN|None, status).

    Output buffers are allocated (flat complex128, sized from out_off + M^2) unless given.
    """
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tab = strip_table(strips)
    dev = onsite.device
    P = probs.P
    need = _out_elems(strips, probs)
    if G1N is None:
        G1N = torch.empty(need, dtype=torch.complex128, device=dev)
    if GN1 is True:
        GN1 = torch.empty(need, dtype=torch.complex128, device=dev)
    if GNN is True:
        GNN = torch.empty(need, dtype=torch.complex128, device=dev)
    GN1 = GN1 if isinstance(GN1, torch.Tensor) else None
    GNN = GNN if isinstance(GNN, torch.Tensor) else None
    status = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)
    wsz = _lib.knit_rgf_sweep_workspace(tab, len(strips), _ptr(probs.host), P, prec, GN1 is not None)
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(max(int(wsz), 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_rgf_sweep(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P, _ptr(_z(onsite)),
                               _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), prec, _ptr(G1N), _ptr(GN1),
                               _ptr(GNN), _ptr(status), _ptr(workspace), workspace.numel(),
                               _stream(stream))
    _check(code, "knit_rgf_sweep")
    return G1N, GN1, GNN, status[:P]


def knit_rgf_sweep_noalloc(strips, probs: ProblemTable, onsite: torch.Tensor, sigmaL: torch.Tensor,
                           sigmaR: torch.Tensor, precision="fp64", G1N: torch.Tensor = None,
                           GN1: torch.Tensor | None = None, GNN: torch.Tensor | None = None,
                           status: torch.Tensor | None = None, stream=None):
    """knit_rgf_sweep with the library's static scratch as work memory: the C call allocates
    nothing.  Outputs and the status word buffer are the caller's (allocated here only when not
    given, before the call).  Returns (G1N, GN1, GNN, status)."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tab = strip_table(strips)
    dev = onsite.device
    P = probs.P
    if G1N is None:
        G1N = torch.empty(_out_elems(strips, probs), dtype=torch.complex128, device=dev)
    if status is None:
        status = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)
    code = _lib.knit_rgf_sweep_noalloc(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P, _ptr(_z(onsite)),
                                       _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), prec, _ptr(G1N), _ptr(GN1), _ptr(GNN),
                                       _ptr(status), _stream(stream))
    _check(code, "knit_rgf_sweep_noalloc")
    return G1N, GN1, GNN, status[:P]


def knit_rgf_sweep_workspace(strips, probs: ProblemTable, precision="fp64", want_gn1=False) -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tab = strip_table(strips)
    return int(_lib.knit_rgf_sweep_workspace(tab, len(strips), _ptr(probs.host), probs.P, prec,
                                             int(want_gn1)))


def knit_transmission(strips, probs: ProblemTable, sigmaL, sigmaR, G1N, GN1=None, GNN=None,
                      stream=None):
    """Returns (T, T_RL|None, T_ward|None) as device float64 [P]."""
    tab = strip_table(strips)
    dev = G1N.device
    P = probs.P
    T = torch.empty(P, dtype=torch.float64, device=dev)
    T_RL = torch.empty(P, dtype=torch.float64, device=dev) if GN1 is not None else None
    T_w = torch.empty(P, dtype=torch.float64, device=dev) if GNN is not None else None
    code = _lib.knit_transmission(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P,
                                  _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), _ptr(G1N), _ptr(GN1), _ptr(GNN),
                                  _ptr(T), _ptr(T_RL), _ptr(T_w), _stream(stream))
    _check(code, "knit_transmission")
    return T, T_RL, T_w


def knit_ldos_workspace(strips, probs: ProblemTable, precision="fp64", checkpoint_stride: int = 0) -> int:
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tab = strip_table(strips)
    return int(_lib.knit_ldos_workspace(tab, len(strips), _ptr(probs.host), probs.P, prec,
                                        int(checkpoint_stride)))


def knit_ldos(strips, probs: ProblemTable, onsite, sigmaL, sigmaR, precision="fp64",
              checkpoint_stride: int = 0, stream=None, workspace: torch.Tensor | None = None):
    """Returns (ldos flat float64 addressed by ldos_off, status [P])."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tab = strip_table(strips)
    dev = onsite.device
    P = probs.P
    n = 0
    for p in probs.host:
        M = _strip_M(strips[int(p["strip"])])
        n = max(n, int(p["ldos_off"]) + int(p["L"]) * M)
    ldos = torch.empty(max(n, 1), dtype=torch.float64, device=dev)
    status = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)
    wsz = _lib.knit_ldos_workspace(tab, len(strips), _ptr(probs.host), P, prec, int(checkpoint_stride))
    ws = workspace
    if ws is None or ws.numel() < wsz:
        ws = torch.empty(max(int(wsz), 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_ldos(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P, _ptr(_z(onsite)),
                          _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), prec, int(checkpoint_stride), _ptr(ldos),
                          _ptr(status), _ptr(ws), int(ws.numel()), _stream(stream))
    _check(code, "knit_ldos")
    return ldos, status[:P]


def knit_gamma_factor(M: int, sigma: torch.Tensor, n: int, tol: float = 0.0, C: torch.Tensor | None = None,
                      stream=None):
    """Gamma = C C^+ factors of n consecutive [M, M] self-energies (complex128 device tensor
    of n*M*M elements, any shape).  Returns (C shaped like sigma, rank [n] int32)."""
    sigma = _z(sigma)
    assert sigma.numel() == n * M * M
    if C is None:
        C = torch.empty_like(sigma)
    assert _z(C).numel() == sigma.numel()
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=sigma.device)
    code = _lib.knit_gamma_factor(int(M), _ptr(sigma), int(n), float(tol), _ptr(C), _ptr(rank), _stream(stream))
    _check(code, "knit_gamma_factor")
    return C, rank[:n]


def knit_rgf_sweep_projected(strips, probs: ProblemTable, onsite, sigmaL, sigmaR, CL, G1Np=None,
                             GNN: torch.Tensor | bool = False, stream=None, workspace: torch.Tensor | None = None,
                             precision="fp64"):
    """Projected sweep: returns (G1Np, GNN|None, status) with P_L = C_L^+ G_1L at out_off."""
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    tab = strip_table(strips)
    dev = onsite.device
    P = probs.P
    need = _out_elems(strips, probs)
    if G1Np is None:
        G1Np = torch.empty(need, dtype=torch.complex128, device=dev)
    if GNN is True:
        GNN = torch.empty(need, dtype=torch.complex128, device=dev)
    GNN = GNN if isinstance(GNN, torch.Tensor) else None
    status = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)
    wsz = _lib.knit_rgf_sweep_workspace(tab, len(strips), _ptr(probs.host), P, prec, 0)
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(max(int(wsz), 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_rgf_sweep_projected(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P,
                                         _ptr(_z(onsite)), _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), _ptr(_z(CL)), prec,
                                         _ptr(G1Np), _ptr(GNN), _ptr(status), _ptr(workspace),
                                         workspace.numel(), _stream(stream))
    _check(code, "knit_rgf_sweep_projected")
    return G1Np, GNN, status[:P]


def knit_transmission_projected(strips, probs: ProblemTable, CR, G1Np, stream=None):
    """T = ||P_L C_R||_F^2 per problem, device float64 [P]."""
    tab = strip_table(strips)
    T = torch.empty(max(probs.P, 1), dtype=torch.float64, device=G1Np.device)
    code = _lib.knit_transmission_projected(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), probs.P,
                                            _ptr(_z(CR)), _ptr(_z(G1Np)), _ptr(T), _stream(stream))
    _check(code, "knit_transmission_projected")
    return T[:probs.P]


def knit_transmission_eigenvalues(strips, probs: ProblemTable, CR, G1Np, stream=None,
                                  workspace: torch.Tensor | None = None):
    """Transmission eigenvalues from the projected propagator.  Returns (tn [P, ld] descending,
    nch [P] int32, T [P], fano [P]) on the device, ld = the largest M of the batch."""
    tab = strip_table(strips)
    dev = G1Np.device
    P = probs.P
    ld = max(1, max((_strip_M(s) for s in strips), default=1))
    tn = torch.empty((max(P, 1), ld), dtype=torch.float64, device=dev)
    nch = torch.empty(max(P, 1), dtype=torch.int32, device=dev)
    T = torch.empty(max(P, 1), dtype=torch.float64, device=dev)
    fano = torch.empty(max(P, 1), dtype=torch.float64, device=dev)
    wsz = int(_lib.knit_transmission_eigenvalues_workspace(tab, len(strips), _ptr(probs.host), P))
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_transmission_eigenvalues(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P, _ptr(_z(CR)),
                                              _ptr(_z(G1Np)), ld, _ptr(tn), _ptr(nch), _ptr(T), _ptr(fano),
                                              _ptr(workspace), workspace.numel(), _stream(stream))
    _check(code, "knit_transmission_eigenvalues")
    return tn[:P], nch[:P], T[:P], fano[:P]


def knit_local_observables(strips, probs: ProblemTable, onsite, sigmaL, sigmaR, CL, checkpoint_stride: int = 0,
                           stream=None, workspace: torch.Tensor | None = None):
    """Injection from the left lead: returns (blk flat complex128 addressed by the returned
    blk_off [P] (host int64), jlong and jtran flat float64 addressed by ldos_off, status [P])."""
    tab = strip_table(strips)
    dev = onsite.device
    P = probs.P
    n_ld, offs, pos = 1, [], 0
    for p in probs.host:
        st = strips[int(p["strip"])]
        M = _strip_M(st)
        n_ld = max(n_ld, int(p["ldos_off"]) + int(p["L"]) * M)
        offs.append(pos)
        pos += int(p["L"]) * M * int(st.norb)
    blk_off = np.array(offs, dtype=np.int64)
    blk = torch.empty(max(pos, 1), dtype=torch.complex128, device=dev)
    blk_off_d = torch.from_numpy(blk_off).to(dev)
    jlong = torch.empty(n_ld, dtype=torch.float64, device=dev)
    jtran = torch.empty(n_ld, dtype=torch.float64, device=dev)
    status = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)
    wsz = int(_lib.knit_local_observables_workspace(tab, len(strips), _ptr(probs.host), P, int(checkpoint_stride)))
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_local_observables(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P, _ptr(_z(onsite)),
                                       _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), _ptr(_z(CL)), int(checkpoint_stride),
                                       _ptr(blk), _ptr(blk_off_d), _ptr(jlong), _ptr(jtran), _ptr(status),
                                       _ptr(workspace), workspace.numel(), _stream(stream))
    _check(code, "knit_local_observables")
    return blk, blk_off, jlong, jtran, status[:P]


LEAD_DTYPE = np.dtype([("slice", "<i4"), ("reserved", "<i4"), ("sigma_off", "<i8")], align=True)
assert LEAD_DTYPE.itemsize == 16
KNIT_MAX_SIDE_LEADS = 6


def knit_conductance_matrix(strips, probs: ProblemTable, onsite, sigmaL, sigmaR, CL, CR, side: np.ndarray,
                            sigmaX=None, CX=None, checkpoint_stride: int = 0, stream=None,
                            workspace: torch.Tensor | None = None):
    """Conductance matrix with side leads.  side: host LEAD_DTYPE [P, n_side] (slice, offsets into
    sigmaX / CX).  Returns (T [P, K, K] float64 with K = n_side + 2, status [P])."""
    tab = strip_table(strips)
    dev = onsite.device
    P = probs.P
    side = np.ascontiguousarray(side, dtype=LEAD_DTYPE).reshape(P, -1)
    n_side = side.shape[1]
    K = n_side + 2
    side_dev = torch.from_numpy(side.view(np.uint8).reshape(-1).copy()).to(dev) if n_side else None
    T = torch.empty((max(P, 1), K, K), dtype=torch.float64, device=dev)
    status = torch.zeros(max(P, 1), dtype=torch.int32, device=dev)
    wsz = int(_lib.knit_conductance_matrix_workspace(tab, len(strips), _ptr(probs.host), P, n_side,
                                                     int(checkpoint_stride)))
    if workspace is None or workspace.numel() < wsz:
        workspace = torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev)
    code = _lib.knit_conductance_matrix(tab, len(strips), _ptr(probs.host), _ptr(probs.dev), P, _ptr(_z(onsite)),
                                        _ptr(_z(sigmaL)), _ptr(_z(sigmaR)), _ptr(_z(CL)), _ptr(_z(CR)), n_side,
                                        _ptr(side) if n_side else None, _ptr(side_dev),
                                        _ptr(sigmaX), _ptr(CX), int(checkpoint_stride), _ptr(T), _ptr(status),
                                        _ptr(workspace), workspace.numel(), _stream(stream))
    _check(code, "knit_conductance_matrix")
    return T[:P], status[:P]


def _strip_M(s) -> int:
    return int(s.M)


def _out_elems(strips, probs: ProblemTable) -> int:
    n = 1
    for p in probs.host:
        M = _strip_M(strips[int(p["strip"])])
        n = max(n, int(p["out_off"]) + M * M)
    return n
