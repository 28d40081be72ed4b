"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function include/knit.h and
include/knit_mlp.h declare, and
reject bad arguments on the host, before any HIP call, with KNIT_E_ARG or
KNIT_E_WORKSPACE.  Device pointers passed here are fake, non-null addresses:
every call below fails validation, so none is ever dereferenced.
"""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1010_2627_amd", "libknit.so")


@pytest.fixture(scope="module")
def K():
    if not os.path.exists(LIB):
        from paper_1010_2627_amd import build
        build.build()
    from paper_1010_2627_amd import knit
    return knit


def _declared(header="knit.h"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(knit_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol(K):
    names = _declared()
    assert len(names) >= 9
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(K.EXPORTED) == names


def test_library_exports_every_sampler_kernel_entry(K):
    from paper_1010_2627_amd import mlp
    names = _declared("knit_mlp.h")
    assert len(names) == 6
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(mlp.EXPORTED) == names


def test_abi_version_and_status_strings(K):
    assert K.abi_version() == 4
    assert K.status_string(K.KNIT_E_ARG) == "invalid argument"
    assert "singular" in K.status_string(K.KNIT_P_SINGULAR)


FAKE = 0x1000   # never dereferenced: validation fails first


def _strip(M=4, norb=1, H0=FAKE, vcol=FAKE, vblk=FAKE):
    from paper_1010_2627_amd.knit import KnitStrip
    return KnitStrip(M, norb, H0, vcol, vblk)


def _probs(rows):
    from paper_1010_2627_amd.knit import PROBLEM_DTYPE
    return np.array(rows, dtype=PROBLEM_DTYPE)


def _sweep(K, strips, probs, **kw):
    arr = (K.KnitStrip * len(strips))(*strips) if strips else None
    a = dict(n=len(strips), pd=FAKE, onsite=FAKE, sL=FAKE, sR=FAKE, prec=0, G1N=FAKE, GN1=None,
             GNN=None, st=FAKE, ws=FAKE, wsb=1 << 40, stream=None)
    a.update(kw)
    ph = probs.ctypes.data if probs is not None and len(probs) else (None if probs is None else probs.ctypes.data)
    return K._lib.knit_rgf_sweep(arr, a["n"], ph, a["pd"], len(probs) if probs is not None else 0,
                                 a["onsite"], a["sL"], a["sR"], a["prec"], a["G1N"], a["GN1"], a["GNN"],
                                 a["st"], a["ws"], a["wsb"], a["stream"])


def test_sweep_rejects_bad_strip_descriptions(K):
    good = _probs([(0, 8, 0.1, 0, 0, 0, 0)])
    assert _sweep(K, [_strip(M=0)], good) == K.KNIT_E_ARG
    assert _sweep(K, [_strip(M=5, norb=2)], good) == K.KNIT_E_ARG          # norb does not divide M
    assert _sweep(K, [_strip(norb=0)], good) == K.KNIT_E_ARG
    assert _sweep(K, [_strip(M=4096)], good) == K.KNIT_E_ARG               # above KNIT_MAX_M
    assert _sweep(K, [_strip(H0=None)], good) == K.KNIT_E_ARG
    assert _sweep(K, [_strip(vcol=None)], good) == K.KNIT_E_ARG
    bad_band = _strip()
    bad_band.h0_band = -1
    assert _sweep(K, [bad_band], good) == K.KNIT_E_ARG
    assert _sweep(K, [], good, n=0) == K.KNIT_E_ARG


def test_h0_band_of_lattice_strips(K):
    """Hard-wall lattice strips have site-block band 1 (nearest transverse neighbours); a band
    that spans the slice, or no coupling at all, states nothing (0)."""
    from paper_1010_2627_amd import inputs
    sq = inputs.square_strip(12)
    assert K.h0_band_of(sq.H0, sq.norb) == 1
    ra = inputs.rashba_strip(8)
    assert K.h0_band_of(ra.H0, ra.norb) == 1
    W = 6
    ring = np.zeros((W, W), dtype=np.complex128)
    for a in range(W):
        ring[a, (a + 1) % W] = ring[(a + 1) % W, a] = -1.0
    assert K.h0_band_of(ring, 1) == 0        # periodic: the corner blocks span the slice
    assert K.h0_band_of(np.eye(W, dtype=np.complex128), 1) == 0


def test_sweep_rejects_bad_problems(K):
    s = [_strip()]
    assert _sweep(K, s, _probs([(1, 8, 0.1, 0, 0, 0, 0)])) == K.KNIT_E_ARG    # strip index
    assert _sweep(K, s, _probs([(0, 0, 0.1, 0, 0, 0, 0)])) == K.KNIT_E_ARG    # L < 1
    assert _sweep(K, s, _probs([(0, 4, np.nan, 0, 0, 0, 0)])) == K.KNIT_E_ARG  # E not finite
    assert _sweep(K, s, _probs([(0, 4, 0.1, -1, 0, 0, 0)])) == K.KNIT_E_ARG   # negative offset
    good = _probs([(0, 4, 0.1, 0, 0, 0, 0)])
    assert _sweep(K, s, good, prec=7) == K.KNIT_E_ARG                           # precision
    assert _sweep(K, s, good, G1N=None) == K.KNIT_E_ARG                         # missing output
    assert _sweep(K, s, good, st=None) == K.KNIT_E_ARG
    assert _sweep(K, s, good, pd=None) == K.KNIT_E_ARG


def test_sweep_workspace_checks(K):
    s = [_strip(M=16)]
    probs = _probs([(0, 8, 0.1, 0, 0, 0, 0), (0, 8, 0.2, 0, 0, 256, 0)])
    arr = (K.KnitStrip * 1)(*s)
    need = K._lib.knit_rgf_sweep_workspace(arr, 1, probs.ctypes.data, 2, 0, 0)
    assert need > 0
    need32 = K._lib.knit_rgf_sweep_workspace(arr, 1, probs.ctypes.data, 2, 2, 0)
    assert 0 < need32 < need
    assert _sweep(K, s, probs, wsb=need - 1) == K.KNIT_E_WORKSPACE
    assert _sweep(K, s, probs, ws=None) == K.KNIT_E_WORKSPACE
    # invalid requests size to 0
    assert K._lib.knit_rgf_sweep_workspace(arr, 1, probs.ctypes.data, 2, 9, 0) == 0


def test_empty_batch_is_ok_without_device(K):
    s = [_strip()]
    assert _sweep(K, s, _probs([])) == K.KNIT_OK


def test_selfenergy_argument_checks(K):
    s = _strip(M=8)
    E = FAKE
    f = K._lib.knit_lead_selfenergy
    ws_need = K._lib.knit_lead_selfenergy_workspace(ctypes.byref(s), 3)
    assert ws_need > 0
    args = lambda **kw: dict(dict(side=0, E=E, nE=3, eta=1e-13, tol=1e-16, it=50, sig=FAKE, iters=None,
                                  st=FAKE, ws=FAKE, wsb=ws_need), **kw)
    def call(**kw):
        a = args(**kw)
        return f(ctypes.byref(s), a["side"], a["E"], a["nE"], a["eta"], a["tol"], a["it"], a["sig"],
                 a["iters"], a["st"], a["ws"], a["wsb"], None)
    assert call(side=3) == K.KNIT_E_ARG
    assert call(side=-1) == K.KNIT_E_ARG
    assert call(eta=0.0) == K.KNIT_E_ARG
    assert call(eta=float("inf")) == K.KNIT_E_ARG
    assert call(tol=-1.0) == K.KNIT_E_ARG
    assert call(it=0) == K.KNIT_E_ARG
    assert call(nE=-1) == K.KNIT_E_ARG
    assert call(sig=None) == K.KNIT_E_ARG
    assert call(E=None) == K.KNIT_E_ARG
    assert call(wsb=ws_need - 1) == K.KNIT_E_WORKSPACE
    assert call(nE=0) == K.KNIT_OK
    big = _strip(M=520)
    assert f(ctypes.byref(big), 0, E, 3, 1e-13, 1e-16, 50, FAKE, None, FAKE, FAKE, 1 << 40, None) \
        == K.KNIT_E_UNSUPPORTED
    bad = _strip(M=6, norb=4)
    assert f(ctypes.byref(bad), 0, E, 3, 1e-13, 1e-16, 50, FAKE, None, FAKE, FAKE, 1 << 40, None) == K.KNIT_E_ARG


def test_transmission_and_ldos_argument_checks(K):
    s = (K.KnitStrip * 1)(_strip())
    probs = _probs([(0, 4, 0.1, 0, 0, 0, 0)])
    t = K._lib.knit_transmission
    assert t(s, 1, probs.ctypes.data, FAKE, 1, FAKE, FAKE, FAKE, None, None, None, None, None, None) == K.KNIT_E_ARG
    # T_RL requested without GN1
    assert t(s, 1, probs.ctypes.data, FAKE, 1, FAKE, FAKE, FAKE, None, None, FAKE, FAKE, None, None) == K.KNIT_E_ARG
    ld = K._lib.knit_ldos
    need = K._lib.knit_ldos_workspace(s, 1, probs.ctypes.data, 1, 0, 0)
    assert need > 0
    assert ld(s, 1, probs.ctypes.data, FAKE, 1, FAKE, FAKE, FAKE, 0, 0, FAKE, FAKE, FAKE, need - 1, None) == K.KNIT_E_WORKSPACE
    assert ld(s, 1, probs.ctypes.data, FAKE, 1, FAKE, FAKE, FAKE, 0, 0, None, FAKE, FAKE, need, None) == K.KNIT_E_ARG


def test_sweep_tuning_table_round_trip(K):
    """The launch-tuning table is host state: validation and set/get need no device."""
    f_set, f_get = K._lib.knit_sweep_tuning_set, K._lib.knit_sweep_tuning_get
    T = K.KnitSweepTuning
    out = T()
    # defaults: 256 threads and two workgroups per unit up to Mp = 256, then 512 threads, one per
    # unit; outer panels of 64 below Mp = 128, else 128
    assert f_get(K.KNIT_FP64, 3, ctypes.byref(out)) == K.KNIT_OK            # Mp = 128
    assert (out.threads, out.wg_per_cu, out.order, out.outer) == (256, 2, 1, 128)
    assert f_get(K.KNIT_FP64, 15, ctypes.byref(out)) == K.KNIT_OK           # Mp = 512
    assert (out.threads, out.wg_per_cu, out.order, out.outer) == (512, 1, 1, 128)
    # bad arguments
    assert f_set(7, 3, ctypes.byref(T(256, 1, 0, 64))) == K.KNIT_E_ARG           # precision
    assert f_set(K.KNIT_FP64, 16, ctypes.byref(T(512, 1, 0, 64))) == K.KNIT_E_ARG  # class
    assert f_set(K.KNIT_FP64, -1, ctypes.byref(T(512, 1, 0, 64))) == K.KNIT_E_ARG
    assert f_set(K.KNIT_FP64, 8, ctypes.byref(T(256, 1, 0, 64))) == K.KNIT_E_ARG   # Mp = 288 > 256 threads
    assert f_set(K.KNIT_FP64, 3, ctypes.byref(T(384, 1, 0, 64))) == K.KNIT_E_ARG
    assert f_set(K.KNIT_FP64, 3, ctypes.byref(T(256, 3, 0, 64))) == K.KNIT_E_ARG
    assert f_set(K.KNIT_FP64, 3, ctypes.byref(T(256, 1, 2, 64))) == K.KNIT_E_ARG
    assert f_set(K.KNIT_FP64, 3, ctypes.byref(T(256, 1, 0, 96))) == K.KNIT_E_ARG   # outer width
    assert f_get(K.KNIT_FP64, 3, None) == K.KNIT_E_ARG
    # round trip, then reset to the default
    assert f_set(K.KNIT_FP32_REFINE, 3, ctypes.byref(T(512, 1, 0, 128))) == K.KNIT_OK
    assert K.knit_sweep_tuning_get("fp32_refine", 3) == {"threads": 512, "wg_per_cu": 1, "order": 0, "outer": 128}
    assert K.knit_sweep_tuning_get("fp64", 3) == {"threads": 256, "wg_per_cu": 2, "order": 1, "outer": 128}
    K.knit_sweep_tuning_set("fp32_refine", 3, None)
    assert K.knit_sweep_tuning_get("fp32_refine", 3) == {"threads": 256, "wg_per_cu": 2, "order": 1, "outer": 128}


def test_autotune_candidates_and_json(K, tmp_path):
    from paper_1010_2627_amd import autotune
    assert all(c["threads"] >= 288 for c in autotune.candidates(288))
    assert len(autotune.candidates(128)) == 16 and len(autotune.candidates(512)) == 8
    assert len(autotune.candidates(64)) == 8                     # no 128-wide outer panel in a 64 slice
    best = {"threads": 512, "wg_per_cu": 1, "order": 0, "outer": 128}
    tuned = [{"precision": "fp64", "cls": 5, "Mp": 192, "best": best, "results": [(best, 0.5)]}]
    path = str(tmp_path / "tuning.json")
    autotune.save(path, tuned)
    try:
        assert autotune.load(path) == 1
        assert K.knit_sweep_tuning_get("fp64", 5) == best
    finally:
        K.knit_sweep_tuning_set("fp64", 5, None)


def test_refine_threshold_validation(K):
    old = K.knit_get_refine_threshold()
    try:
        assert K._lib.knit_set_refine_threshold(-1.0) == K.KNIT_E_ARG
        assert K._lib.knit_set_refine_threshold(float("nan")) == K.KNIT_E_ARG
        assert K._lib.knit_set_refine_threshold(0.0) == K.KNIT_OK
        assert K.knit_get_refine_threshold() == 0.0
        assert K._lib.knit_set_refine_threshold(float("inf")) == K.KNIT_OK
        K.knit_set_refine_threshold(0.25)
        assert K.knit_get_refine_threshold() == 0.25
    finally:
        K.knit_set_refine_threshold(old)
    assert K.status_string(K.KNIT_P_FALLBACK).startswith("refinement")


def test_sampler_kernel_argument_checks(K):
    lib = K._lib
    from paper_1010_2627_amd import mlp  # noqa: F401  (sets the argument types)
    assert lib.knit_mlp_gemm(-1, 4, 4, FAKE, 4, 1, FAKE, 4, 1, None, 0.0, FAKE, 4, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_gemm(4, 4, 4, FAKE, 4, 1, FAKE, 4, 1, None, 0.0, FAKE, 3, None) == K.KNIT_E_ARG   # ldc < N
    assert lib.knit_mlp_gemm(4, 4, 4, None, 4, 1, FAKE, 4, 1, None, 0.0, FAKE, 4, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_gemm(0, 4, 4, None, 4, 1, None, 4, 1, None, 0.0, None, 4, None) == K.KNIT_OK
    assert lib.knit_mlp_act_fwd(-1, FAKE, FAKE, 1, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_act_fwd(0, None, None, 1, None) == K.KNIT_OK
    assert lib.knit_mlp_gelu_bwd(4, FAKE, None, FAKE, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_softmax_xent(4, 8, None, FAKE, 1.0, FAKE, None, None, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_softmax_xent(4, 8, FAKE, None, 1.0, FAKE, None, None, None) == K.KNIT_E_ARG  # loss needs q
    assert lib.knit_mlp_colsum(4, 8, None, FAKE, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_adamw(4, FAKE, None, FAKE, FAKE, FAKE, 1e-3, 1.0, 0.99, 1e-8, 0.0, 1, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_adamw(4, FAKE, None, FAKE, FAKE, FAKE, 1e-3, 0.9, 0.99, 1e-8, 0.0, 0, None) == K.KNIT_E_ARG
    assert lib.knit_mlp_adamw(4, FAKE, None, None, FAKE, FAKE, 1e-3, 0.9, 0.99, 1e-8, 0.0, 1, None) == K.KNIT_E_ARG


def test_projected_path_argument_checks(K):
    lib = K._lib
    # Gamma factors
    assert lib.knit_gamma_factor(0, FAKE, 2, 0.0, FAKE, FAKE, None) == K.KNIT_E_ARG
    assert lib.knit_gamma_factor(4096, FAKE, 2, 0.0, FAKE, FAKE, None) == K.KNIT_E_ARG    # above KNIT_MAX_M
    assert lib.knit_gamma_factor(8, FAKE, -1, 0.0, FAKE, FAKE, None) == K.KNIT_E_ARG
    assert lib.knit_gamma_factor(8, FAKE, 2, float("nan"), FAKE, FAKE, None) == K.KNIT_E_ARG
    assert lib.knit_gamma_factor(8, None, 2, 0.0, FAKE, FAKE, None) == K.KNIT_E_ARG
    assert lib.knit_gamma_factor(8, FAKE, 2, 0.0, FAKE, None, None) == K.KNIT_E_ARG
    assert lib.knit_gamma_factor(8, None, 0, 0.0, None, None, None) == K.KNIT_OK
    # projected sweep: FP64 matrix-core path only, the FP64 sweep's workspace
    s = (K.KnitStrip * 1)(_strip(M=16))
    probs = _probs([(0, 8, 0.1, 0, 0, 0, 0), (0, 8, 0.2, 0, 0, 256, 0)])
    need = lib.knit_rgf_sweep_workspace(s, 1, probs.ctypes.data, 2, 0, 0)
    sw = lambda **kw: lib.knit_rgf_sweep_projected(
        s, 1, probs.ctypes.data, FAKE, 2, FAKE, FAKE, FAKE, kw.get("CL", FAKE), kw.get("prec", 0),
        kw.get("G1Np", FAKE), None, FAKE, kw.get("ws", FAKE), kw.get("wsb", need), None)
    assert sw(CL=None) == K.KNIT_E_ARG
    assert sw(prec=5) == K.KNIT_E_ARG
    # the refined projected sweep needs the refined workspace (its FP64 second pass shares it)
    need_r = lib.knit_rgf_sweep_workspace(s, 1, probs.ctypes.data, 2, 1, 0)
    assert need_r >= need
    assert sw(prec=1, wsb=need_r - 1) == K.KNIT_E_WORKSPACE
    assert sw(G1Np=None) == K.KNIT_E_ARG
    assert sw(wsb=need - 1) == K.KNIT_E_WORKSPACE
    assert sw(ws=None) == K.KNIT_E_WORKSPACE
    wide = (K.KnitStrip * 1)(_strip(M=544))
    assert lib.knit_rgf_sweep_projected(wide, 1, probs.ctypes.data, FAKE, 2, FAKE, FAKE, FAKE, FAKE, 0, FAKE, None,
                                        FAKE, FAKE, 1 << 40, None) == K.KNIT_E_UNSUPPORTED
    assert lib.knit_rgf_sweep_projected(s, 1, None, None, 0, None, None, None, None, 0, None, None, None, None, 0,
                                        None) == K.KNIT_OK
    # projected transmission
    tp = lib.knit_transmission_projected
    assert tp(s, 1, probs.ctypes.data, FAKE, 2, None, FAKE, FAKE, None) == K.KNIT_E_ARG
    assert tp(s, 1, probs.ctypes.data, FAKE, 2, FAKE, FAKE, None, None) == K.KNIT_E_ARG
    assert tp(s, 1, _probs([(0, 0, 0.1, 0, 0, 0, 0)]).ctypes.data, FAKE, 1, FAKE, FAKE, FAKE, None) == K.KNIT_E_ARG


def test_observable_entry_points_argument_checks(K):
    """Transmission eigenvalues, local observables and the conductance matrix reject bad
    arguments before any device call (fake device pointers are never dereferenced)."""
    lib = K._lib
    s = (K.KnitStrip * 1)(_strip(M=16))
    probs = _probs([(0, 8, 0.1, 0, 0, 0, 0), (0, 8, 0.2, 0, 0, 256, 128)])
    ph = probs.ctypes.data
    # transmission eigenvalues
    te = lambda **kw: lib.knit_transmission_eigenvalues(
        s, 1, ph, FAKE, 2, kw.get("CR", FAKE), kw.get("G1Np", FAKE), kw.get("ld", 16), kw.get("tn", FAKE), None,
        None, None, kw.get("ws", FAKE), kw.get("wsb", 1 << 40), None)
    assert te(CR=None) == K.KNIT_E_ARG
    assert te(G1Np=None) == K.KNIT_E_ARG
    assert te(tn=None) == K.KNIT_E_ARG
    assert te(ld=15) == K.KNIT_E_ARG                    # ld below the largest M
    assert te(ws=None) == K.KNIT_E_WORKSPACE
    need = lib.knit_transmission_eigenvalues_workspace(s, 1, ph, 2)
    assert need > 0 and te(wsb=need - 1) == K.KNIT_E_WORKSPACE
    assert lib.knit_transmission_eigenvalues(s, 1, None, None, 0, None, None, 16, None, None, None, None, None, 0,
                                             None) == K.KNIT_OK
    # local observables
    lo = lambda **kw: lib.knit_local_observables(
        s, 1, ph, FAKE, 2, FAKE, FAKE, FAKE, kw.get("CL", FAKE), 0, kw.get("blk", FAKE), FAKE, FAKE, FAKE, FAKE,
        kw.get("ws", FAKE), kw.get("wsb", 1 << 40), None)
    assert lo(CL=None) == K.KNIT_E_ARG
    assert lo(blk=None) == K.KNIT_E_ARG
    assert lo(ws=None) == K.KNIT_E_WORKSPACE
    need = lib.knit_local_observables_workspace(s, 1, ph, 2, 0)
    assert need > 0 and lo(wsb=need - 1) == K.KNIT_E_WORKSPACE
    wide = (K.KnitStrip * 1)(_strip(M=544))
    assert lib.knit_local_observables(wide, 1, ph, FAKE, 2, FAKE, FAKE, FAKE, FAKE, 0, FAKE, FAKE, FAKE, FAKE, FAKE,
                                      FAKE, 1 << 40, None) == K.KNIT_E_UNSUPPORTED
    # conductance matrix: side leads on valid slices only, at most KNIT_MAX_SIDE_LEADS
    from paper_1010_2627_amd.knit import LEAD_DTYPE
    side = np.zeros(2, dtype=LEAD_DTYPE)
    side["slice"] = [3, 5]
    cm = lambda **kw: lib.knit_conductance_matrix(
        s, 1, ph, FAKE, 2, FAKE, FAKE, FAKE, FAKE, FAKE, kw.get("n_side", 1), kw.get("side", side.ctypes.data),
        kw.get("side_dev", FAKE), FAKE, FAKE, 0, kw.get("T", FAKE), FAKE, kw.get("ws", FAKE),
        kw.get("wsb", 1 << 40), None)
    assert cm(n_side=-1) == K.KNIT_E_ARG
    assert cm(n_side=7) == K.KNIT_E_ARG
    assert cm(side_dev=None) == K.KNIT_E_ARG
    assert cm(T=None) == K.KNIT_E_ARG
    bad = side.copy()
    bad["slice"] = [3, 8]                               # slice 8 is past L = 8
    assert cm(side=bad.ctypes.data) == K.KNIT_E_ARG
    assert cm(ws=None) == K.KNIT_E_WORKSPACE
    need = lib.knit_conductance_matrix_workspace(s, 1, ph, 2, 1, 0)
    assert need > 0 and cm(wsb=need - 1) == K.KNIT_E_WORKSPACE


# ---------------------------------------------------------------- knitting of systems of any shape

def test_library_exports_every_graph_entry(K):
    from paper_1010_2627_amd import graph as GR
    names = _declared("knit_graph.h")
    assert len(names) == 7
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(GR.EXPORTED) == names


def _rect(Lx, Ly, **kw):
    from paper_1010_2627_amd import inputs
    g = inputs.square_lattice_graph(inputs.rectangle_with_hole(Lx, Ly), **kw)
    idx = {s: i for i, s in enumerate(g.coords)}
    left = [idx[(0, y)] for y in range(Ly)]
    right = [idx[(Lx - 1, y)] for y in range(Ly)]
    return g, left, right


def test_graph_plan_of_a_rectangle(K):
    """W x L rectangle, leads on the end columns, default (breadth-first) order: lead 0 first,
    every later site touches an earlier one, the interface never exceeds the lead plus one
    column plus the new site, and the step count is N minus lead 0."""
    from paper_1010_2627_amd import graph as GR
    Lx, W = 17, 9
    g, left, right = _rect(Lx, W)
    p = GR.plan_create(g.N, 1, g.row_ptr, g.col, [left, right])
    inf = p.info()
    assert inf["nsite"] == Lx * W and inf["n_steps"] == Lx * W - W
    assert inf["lead_dim"] == 2 * W and inf["sigma_size"] == 2 * W * W
    assert inf["dim"] == 2 * W + 1
    assert inf["nnz"] == 2 * ((Lx - 1) * W + Lx * (W - 1))
    order = p.order()
    assert sorted(order) == list(range(g.N)) and list(order[:W]) == left
    pos = np.empty(g.N, dtype=int)
    pos[order] = np.arange(g.N)
    for t in range(W, g.N):
        i = order[t]
        nb = g.col[g.row_ptr[i]:g.row_ptr[i + 1]]
        assert (pos[nb] < t).any()
    # the update cost is sum over steps of 8 D_t^2 with W + 1 <= D_t <= 2W + 1
    assert 8 * (W + 1) ** 2 * inf["n_steps"] <= inf["update_flops"] <= 8 * (2 * W + 1) ** 2 * inf["n_steps"]
    assert inf["update_bytes"] == 4 * inf["update_flops"]


def test_graph_plan_given_order_and_norb(K):
    from paper_1010_2627_amd import graph as GR
    g, left, right = _rect(6, 4, kind="bdg", mu=0.2, delta=0.1)
    order = np.arange(g.N)[::-1]
    p = GR.plan_create(g.N, 2, g.row_ptr, g.col, [left, right], order)
    o = p.order()
    assert list(o[:4]) == left
    rest = [int(s) for s in order if s not in left]
    assert list(o[4:]) == rest
    assert p.info()["lead_dim"] == 16


def test_graph_plan_rejects_bad_input(K):
    from paper_1010_2627_amd import graph as GR
    g, left, right = _rect(5, 3)
    ok = GR.GraphPlan(g.N, 1, g.row_ptr, g.col, [left, right])
    assert ok.ok()
    # asymmetric structure: drop one direction of the first bond
    rp, col = g.row_ptr.copy(), g.col.copy()
    j = col[0]
    row_j = list(col[rp[j]:rp[j + 1]])
    k = rp[j] + row_j.index(0)
    col2 = np.delete(col, k)
    rp2 = rp.copy()
    rp2[j + 1:] -= 1
    assert GR.GraphPlan(g.N, 1, rp2, col2, [left, right]).code == K.KNIT_E_ARG
    # self loop
    col3 = col.copy()
    col3[0] = 0
    assert GR.GraphPlan(g.N, 1, rp, col3, [left, right]).code == K.KNIT_E_ARG
    # neighbour out of range
    col4 = col.copy()
    col4[0] = g.N
    assert GR.GraphPlan(g.N, 1, rp, col4, [left, right]).code == K.KNIT_E_ARG
    # leads: shared site, site out of range, empty lead
    assert GR.GraphPlan(g.N, 1, rp, col, [left, [left[0]] + right]).code == K.KNIT_E_ARG
    assert GR.GraphPlan(g.N, 1, rp, col, [left, [g.N]]).code == K.KNIT_E_ARG
    assert GR.GraphPlan(g.N, 1, rp, col, [left, []]).code == K.KNIT_E_ARG
    # order: repeated site
    bad = np.arange(g.N)
    bad[1] = 0
    assert GR.GraphPlan(g.N, 1, rp, col, [left, right], bad).code == K.KNIT_E_ARG
    # norb out of range
    assert GR.GraphPlan(g.N, 0, rp, col, [left, right]).code == K.KNIT_E_ARG
    assert GR.GraphPlan(g.N, 5, rp, col, [left, right]).code == K.KNIT_E_ARG


def test_blocked_graph_plan_of_a_rectangle(K):
    """Groups of b sites: the leads' sites b at a time, the others b at a time in the site order.
    The plan keeps the system's sizes (sites, orbitals, edges, lead block, self-energy pack) and
    counts groups for the steps; block 1 is the site-by-site plan; automatic picks the largest
    group that divides every lead and keeps the interface in registers."""
    from paper_1010_2627_amd import graph as GR
    Lx, W = 17, 8
    g, left, right = _rect(Lx, W)
    one = GR.plan_create(g.N, 1, g.row_ptr, g.col, [left, right])
    i1 = one.info()
    same = GR.plan_create(g.N, 1, g.row_ptr, g.col, [left, right], block=1).info()
    assert same == i1 and i1["block"] == 1
    for b in (2, 4):
        p = GR.plan_create(g.N, 1, g.row_ptr, g.col, [left, right], block=b)
        inf = p.info()
        assert inf["block"] == b and inf["nsite"] == g.N and inf["norb"] == 1 and inf["nnz"] == i1["nnz"]
        assert inf["lead_dim"] == i1["lead_dim"] and inf["sigma_size"] == i1["sigma_size"]
        ngroups = -(-(g.N - 2 * W) // b) + 2 * W // b
        assert inf["n_steps"] == ngroups - W // b
        assert inf["dim"] % b == 0 and inf["dim"] >= i1["dim"] - 1
        assert list(p.order()) == list(one.order())
        # the groups' blocks take (P * groups + group edges) * b^2 elements more workspace
        assert p.workspace(3) > one.workspace(3)
    # automatic: groups of 2 one-orbital sites while the interface fits in registers ...
    auto = GR.plan_create(g.N, 1, g.row_ptr, g.col, [left, right], block=0)
    assert auto.info()["block"] == 2 and auto.info()["dim"] <= 64
    g5, l5, r5 = _rect(17, 5)                      # 2 does not divide the leads: site by site
    assert GR.plan_create(g5.N, 1, g5.row_ptr, g5.col, [l5, r5], block=0).info()["block"] == 1
    # ... above, groups of 3 sites where 3 divides the leads, else 4, else 2
    gw, lw, rw = _rect(12, 81)
    assert GR.plan_create(gw.N, 1, gw.row_ptr, gw.col, [lw, rw]).info()["dim"] > 128
    assert GR.plan_create(gw.N, 1, gw.row_ptr, gw.col, [lw, rw], block=0).info()["block"] == 3
    gw, lw, rw = _rect(12, 80)
    assert GR.plan_create(gw.N, 1, gw.row_ptr, gw.col, [lw, rw], block=0).info()["block"] == 4
    gw, lw, rw = _rect(12, 82)
    assert GR.plan_create(gw.N, 1, gw.row_ptr, gw.col, [lw, rw], block=0).info()["block"] == 2
    # two orbitals per site: groups of 2 sites (4 orbitals) with the interface in memory, site
    # by site with it in registers
    gb, lb, rb = _rect(12, 70, kind="bdg", mu=0.2, delta=0.1)
    assert GR.plan_create(gb.N, 2, gb.row_ptr, gb.col, [lb, rb], block=0).info()["block"] == 2
    gb, lb, rb = _rect(8, 6, kind="bdg", mu=0.2, delta=0.1)
    assert GR.plan_create(gb.N, 2, gb.row_ptr, gb.col, [lb, rb], block=0).info()["block"] == 1


def test_blocked_graph_plan_rejects_bad_blocks(K):
    from paper_1010_2627_amd import graph as GR
    g, left, right = _rect(7, 6)
    assert GR.GraphPlan(g.N, 1, g.row_ptr, g.col, [left, right], block=-1).code == K.KNIT_E_ARG
    assert GR.GraphPlan(g.N, 1, g.row_ptr, g.col, [left, right], block=4).code == K.KNIT_E_ARG   # 4 does not divide 6
    assert GR.GraphPlan(g.N, 1, g.row_ptr, g.col, [left, right], block=5).code == K.KNIT_E_ARG   # 5 orbitals per group
    gb, lb, rb = _rect(6, 4, kind="bdg", mu=0.2, delta=0.1)
    assert GR.GraphPlan(gb.N, 2, gb.row_ptr, gb.col, [lb, rb], block=4).code == K.KNIT_E_ARG     # 8 orbitals
    # the site-by-site checks still come first
    col3 = g.col.copy()
    col3[0] = 0
    assert GR.GraphPlan(g.N, 1, g.row_ptr, col3, [left, right], block=2).code == K.KNIT_E_ARG
    # a lead whose sites do not divide: automatic falls back to site by site
    g5, l5, r5 = _rect(6, 5)
    assert GR.plan_create(g5.N, 1, g5.row_ptr, g5.col, [l5, r5], block=0).info()["block"] == 1


def test_blocked_plans_of_random_graphs(K):
    """Random connected graphs (degree <= 4), random leads and orders, every block size: the
    plan is made or refused with an argument or support code, and a plan keeps the system's
    sizes, counts steps of whole groups, and knits every site once."""
    from paper_1010_2627_amd import graph as GR, inputs
    for seed in range(12):
        rng = np.random.Generator(np.random.PCG64(900 + seed))
        N, m = int(rng.integers(20, 60)), int(rng.integers(1, 3))
        perm = rng.permutation(N)
        bonds = {(int(a), int(b)): np.eye(m) for a, b in zip(perm[:-1], perm[1:])}
        deg = np.bincount(np.array(list(bonds)).ravel(), minlength=N)
        for _ in range(N // 3):
            a, b = (int(x) for x in rng.integers(0, N, 2))
            if a != b and deg[a] < 4 and deg[b] < 4 and (a, b) not in bonds and (b, a) not in bonds:
                bonds[(a, b)] = np.eye(m)
                deg[a] += 1
                deg[b] += 1
        g = inputs.graph_from_blocks(N, m, np.zeros((N, m, m)), bonds)
        sizes = [int(x) for x in rng.choice([2, 4, 6], size=int(rng.integers(1, 4)))]
        pick = rng.permutation(N)
        leads, o = [], 0
        for s in sizes:
            leads.append([int(x) for x in pick[o:o + s]])
            o += s
        order = rng.permutation(N) if seed % 2 else None
        ref = GR.GraphPlan(N, m, g.row_ptr, g.col, leads, order)
        assert ref.ok(), (seed, ref.code)
        r = ref.info()
        for block in (0, 1, 2, 3, 4):
            p = GR.GraphPlan(N, m, g.row_ptr, g.col, leads, order, block=block)
            if not p.ok():
                assert p.code in (K.KNIT_E_ARG, K.KNIT_E_UNSUPPORTED), (seed, block, p.code)
                assert block >= 2
                continue
            inf = p.info()
            b = inf["block"]
            assert b == block or block == 0, (seed, block, b)
            assert inf["nsite"] == N and inf["norb"] == m and inf["nnz"] == r["nnz"]
            assert inf["lead_dim"] == r["lead_dim"] and inf["sigma_size"] == r["sigma_size"]
            assert inf["dim"] % (b * m) == 0 and inf["max_pairs"] <= 16
            groups = sum(len(l) // b for l in leads) + -(-(N - sum(sizes)) // b)
            assert inf["n_steps"] == groups - len(leads[0]) // b
            assert sorted(p.order()) == list(range(N))
            assert p.workspace(5) >= ref.workspace(5) or b == 1


def test_graph_plan_refuses_too_many_coupled_orbitals(K):
    """A site joining 5 earlier neighbours with 4 orbitals each couples 20 > 16 orbitals."""
    from paper_1010_2627_amd import graph as GR, inputs
    N, m = 6, 4
    bonds = {(0, 5): np.eye(m), (1, 5): np.eye(m), (2, 5): np.eye(m), (3, 5): np.eye(m), (4, 5): np.eye(m),
             (0, 1): np.eye(m), (1, 2): np.eye(m), (2, 3): np.eye(m), (3, 4): np.eye(m)}
    g = inputs.graph_from_blocks(N, m, np.zeros((N, m, m)), bonds)
    p = GR.GraphPlan(N, m, g.row_ptr, g.col, [[0], [4]], order=np.arange(N))
    assert p.code == K.KNIT_E_UNSUPPORTED


def test_graph_transmission_validates_before_any_device_call(K):
    from paper_1010_2627_amd import graph as GR
    g, left, right = _rect(5, 3)
    p = GR.plan_create(g.N, 1, g.row_ptr, g.col, [left, right])
    L = GR._lib
    assert L.knit_graph_transmission(None, FAKE, 1, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, 1 << 40,
                                     None) == K.KNIT_E_ARG
    assert L.knit_graph_transmission(p.handle, FAKE, -1, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE, 1 << 40,
                                     None) == K.KNIT_E_ARG
    assert L.knit_graph_transmission(p.handle, None, 0, None, None, None, None, None, None, None, 0,
                                     None) == K.KNIT_OK          # empty batch: nothing to do
    assert L.knit_graph_transmission(p.handle, FAKE, 1, None, FAKE, FAKE, FAKE, None, FAKE, FAKE, 1 << 40,
                                     None) == K.KNIT_E_ARG
    assert L.knit_graph_transmission(p.handle, FAKE, 1, FAKE, FAKE, FAKE, FAKE, None, FAKE, None, 1 << 40,
                                     None) == K.KNIT_E_WORKSPACE
    assert L.knit_graph_transmission(p.handle, FAKE, 1, FAKE, FAKE, FAKE, FAKE, None, FAKE, FAKE,
                                     p.workspace(1) - 1, None) == K.KNIT_E_WORKSPACE
    assert p.workspace(2000) == p.workspace(1024) > p.workspace(1) > 0   # resident workgroups are capped
