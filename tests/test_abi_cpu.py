"""Host-side checks of the HIP library that need no GPU: the shared library
loads and exports every function include/mlsdc_sh.h declares, argument
validation returns the documented codes before touching the device, and the
quad-precision host set-up agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlsdc_sh.h")

pk = pytest.importorskip("paper_1805_07923_amd")
if not os.path.exists(pk.LIB_PATH):
    pytest.skip("libmlsdc_sh.so not built", allow_module_level=True)


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s+\**([a-z_][a-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declarations_exported():
    names = declared_functions()
    assert len(names) >= 19
    L = ctypes.CDLL(pk.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(pk.EXPORTS)


def test_argument_validation_without_device():
    L = pk.lib()
    h = ctypes.c_void_p()
    assert L.shx_plan_create(31, 48, 96, 0, 0, None) == -1
    assert L.shx_plan_create(0, 48, 96, 0, 0, ctypes.byref(h)) == -1
    assert L.shx_plan_create(31, 47, 96, 0, 0, ctypes.byref(h)) == -2     # odd nlat
    assert L.shx_plan_create(31, 48, 62, 0, 0, ctypes.byref(h)) == -2     # nlon <= 2N
    assert L.shx_plan_create(31, 30, 96, 0, 0, ctypes.byref(h)) == -2     # nlat <= N
    assert L.shx_plan_create(31, 48, 100, 0, 0, ctypes.byref(h)) == -3    # not 2^k or 3*2^k
    assert L.shx_plan_create(31, 48, 96, 7, 0, ctypes.byref(h)) == -3     # unknown precision
    assert L.shx_plan_create(7, 12, 24, 0, 0, ctypes.byref(h)) == -3      # 3*2^k below the smallest row (48)
    assert L.shx_plan_create(3, 4, 8, 0, 0, ctypes.byref(h)) == -3        # 2^k below the smallest row (16)
    assert L.shx_plan_create(31, 48, 96, 0, 2, ctypes.byref(h)) == -1  # unknown table mode
    assert L.shx_nspec(31) == 32 * 33 // 2
    assert L.shx_strerror(-4).decode().startswith("workspace")
    par = pk.swe_params()
    assert L.sdc_level_create(None, ctypes.byref(par), 0, 3, ctypes.byref(h)) == -1
    assert L.sh_inverse(None, 1, None, None, None, 0, None) == -1
    assert L.shx_plan_analysis_terms(None, 31, None, None) == -1
    assert L.mlsdc_step(None, None, None, 1.0, None, None, None, None, 0, None) == -1
    assert L.mlsdc_step_noalloc(None, None, None, 1.0, None, None, None, None) == -1


def test_host_gauss_matches_oracle(oracle_gauss):
    L = ctypes.CDLL(pk.LIB_PATH)
    for J in (48, 192, 384, 768, 1536):             # up to the T1023 grid's latitudes
        mu, st, c2, w = (np.empty(J) for _ in range(4))
        assert L.shx_host_gauss(J, mu.ctypes.data_as(ctypes.c_void_p), st.ctypes.data_as(ctypes.c_void_p),
                                c2.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p)) == 0
        omu, ost, oc2, ow = oracle_gauss(J)
        # both are correctly rounded from >= 34-digit values: equal to the last bit or one ulp
        assert np.all(np.abs(mu - omu) <= np.spacing(np.abs(omu)) + 1e-300)
        assert np.all(np.abs(st - ost) <= np.spacing(ost))
        assert np.all(np.abs(w - ow) <= np.spacing(ow))


@pytest.mark.parametrize("kind,nn", [(0, 2), (0, 3), (0, 5), (1, 3), (1, 4), (1, 6)])
def test_host_sdc_matrices_match_oracle(kind, nn):
    from oracle.quadrature import sdc_matrices, transfer_matrix
    L = ctypes.CDLL(pk.LIB_PATH)
    tau, Q, QE, QD = np.empty(nn), np.empty((nn, nn)), np.empty((nn, nn)), np.empty((nn, nn))
    vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    assert L.shx_host_sdc(kind, nn, vp(tau), vp(Q), vp(QE), vp(QD)) == 0
    o = sdc_matrices("lobatto" if kind == 0 else "radau", nn)
    assert np.abs(tau - o.tau).max() <= 2e-16
    assert np.abs(Q - o.Q).max() <= 4e-16
    assert np.abs(QE - o.QE).max() <= 2e-16
    assert np.abs(QD - o.QD).max() <= 4e-16
    if nn >= 3:
        small = nn - 1 if kind == 1 else (nn + 1) // 2
        if kind == 0 and nn == 5:
            small = 3
        Pi = np.empty((small, nn))
        assert L.shx_host_transfer(kind, nn, small, vp(Pi)) == 0
        so = sdc_matrices("lobatto" if kind == 0 else "radau", small)
        assert np.abs(Pi - transfer_matrix(o, so)).max() <= 1e-15
