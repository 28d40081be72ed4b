"""The decimation's double-double products on the INT8 matrix cores (digit planes)
against the same products on the vector units, and both against the oracle.

Both modes must give the leads' self-energies to the accuracy the parity tests
hold them to (1e-11 against the Bloch-mode oracle); against each other they
agree far closer, since both carry about 2^-105 per product.
"""

import numpy as np
import pytest
import torch

from paper_1010_2627_amd import inputs

gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def _sigmas(strip, E, mode):
    from paper_1010_2627_amd import knit as K
    old = K.knit_get_selfenergy_products()
    K.knit_set_selfenergy_products(mode)
    try:
        ds = K.DeviceStrip.from_host(strip, "cuda")
        Et = torch.as_tensor(np.asarray(E, dtype=np.float64), device="cuda")
        sig, it, st = K.knit_lead_selfenergy(ds, 2, Et)
        torch.cuda.synchronize()
        return sig.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()
    finally:
        K.knit_set_selfenergy_products(old)


@pytest.mark.gpu
@gpu
@pytest.mark.parametrize("name", ["square16", "rashba24", "zigzag8", "square61"])
def test_int8_products_match_vector_products_and_oracle(name):
    from oracle import leads as OL
    from paper_1010_2627_amd import knit as K
    st = {"square16": lambda: inputs.square_strip(16), "rashba24": lambda: inputs.rashba_strip(24),
          "zigzag8": lambda: inputs.zigzag_strip(8), "square61": lambda: inputs.square_strip(61)}[name]()
    E = inputs.midpoint_grid(-3.7, 3.7, 8)
    s8, st8, it8 = _sigmas(st, E, K.KNIT_PRODUCTS_INT8)
    sv, stv, itv = _sigmas(st, E, K.KNIT_PRODUCTS_VECTOR)
    assert (st8 == 0).all() and (stv == 0).all(), (st8, stv)
    scale = np.abs(sv).max()
    assert np.abs(s8 - sv).max() <= 1e-12 * scale, np.abs(s8 - sv).max() / scale
    V = st.V_dense()
    for k, e in enumerate(E):
        for side, lbl in ((0, "L"), (1, "R")):
            ref = OL.sigma_modes(st.H0, V, e, lbl)
            assert np.abs(s8[side, k] - ref).max() <= 1e-11 * max(1.0, np.abs(ref).max()), (name, e, lbl)


def test_products_mode_switch():
    from paper_1010_2627_amd import knit as K
    old = K.knit_get_selfenergy_products()
    try:
        for m in (K.KNIT_PRODUCTS_VECTOR, K.KNIT_PRODUCTS_INT8):
            K.knit_set_selfenergy_products(m)
            assert K.knit_get_selfenergy_products() == m
        assert K._lib.knit_set_selfenergy_products(2) == K.KNIT_E_ARG
        assert K._lib.knit_set_selfenergy_products(-1) == K.KNIT_E_ARG
    finally:
        K.knit_set_selfenergy_products(old)


@pytest.mark.gpu
@gpu
def test_slice_eigenvalue_energies_still_recovered():
    """E = 0 on the zigzag lead and on an odd-width square lead are slice eigenvalues:
    the first pass fails its check and the two-slice-cell retry (vector products)
    recovers them, with the INT8 products enabled as with them disabled."""
    from oracle import leads as OL
    from paper_1010_2627_amd import knit as K
    for st in (inputs.zigzag_strip(8), inputs.square_strip(15)):
        E = np.array([0.0, 0.6])
        s8, st8, _ = _sigmas(st, E, K.KNIT_PRODUCTS_INT8)
        sv, stv, _ = _sigmas(st, E, K.KNIT_PRODUCTS_VECTOR)
        assert (st8 == stv).all(), (st8, stv)
        ok = st8 == 0
        assert ok[1]
        assert np.abs(s8[:, ok] - sv[:, ok]).max() <= 1e-11 * np.abs(sv[:, ok]).max()
