"""CPU-side checks of the C-ABI library: it loads and exports every symbol declared
in include/psms.h, and argument errors are reported without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psms.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psms_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["psms_create", "psms_destroy", "psms_gauge_load", "psms_apply_dw", "psms_apply_block",
              "psms_apply_hop_bw", "psms_apply_proj", "psms_solve", "psms_solve_block", "psms_apply_schur",
              "psms_apply_schur_inv", "psms_logdet_ratio"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1204_1306_amd import psms

    if not os.path.exists(psms.LIB_PATH):
        pytest.skip("libpsms.so not built")
    lib = ctypes.CDLL(psms.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for every exported function of the header
    assert set(declared_functions()) <= set(psms._SIGS)


def test_null_and_bad_arguments_are_rejected_on_the_host():
    from paper_1204_1306_amd import psms

    if not os.path.exists(psms.LIB_PATH):
        pytest.skip("libpsms.so not built")
    lib = psms.load_library()
    assert lib.psms_create(None, 0, None, None) == -1
    assert lib.psms_apply_dw(None, 0, None, None, 1, 0) == -1
    assert lib.psms_status_string(-4) == b"solver did not converge"
    p = psms.default_params()
    assert p.tol == 1e-10 and p.restart == 16 and p.pc == psms.PC_SAP


@pytest.mark.parametrize("L,b,sap_b,kappa", [
    ((8, 8, 8, 8), (3, 4, 4, 4), (0, 0, 0, 0), 0.15),   # L not a multiple of b
    ((8, 8, 8, 8), (4, 4, 4, 8), (0, 0, 0, 0), 0.15),   # L/b odd in direction 3 (inconsistent colouring)
    ((6, 6, 6, 6), (3, 3, 3, 3), (0, 0, 0, 0), 0.15),   # odd block extent (no even-odd order inside blocks)
    ((8, 8, 8, 8), (4, 4, 4, 4), (0, 0, 0, 0), -0.1),   # negative kappa
    ((8, 8, 8, 8), (4, 4, 4, 4), (2, 2, 2, 3), 0.15),   # Schwarz block does not divide the block
    ((0, 8, 8, 8), (4, 4, 4, 4), (0, 0, 0, 0), 0.15),   # empty lattice
])
def test_bad_geometries_are_rejected_before_any_device_work(L, b, sap_b, kappa):
    from paper_1204_1306_amd import psms

    if not os.path.exists(psms.LIB_PATH):
        pytest.skip("libpsms.so not built")
    lib = psms.load_library()
    g = psms.Geom()
    for m in range(4):
        g.L[m], g.b[m], g.sap_b[m] = L[m], b[m], sap_b[m]
    g.antiperiodic_t = 1
    g.kappa = kappa
    out = ctypes.c_void_p()
    assert lib.psms_create(ctypes.byref(g), 0, None, ctypes.byref(out)) == -1  # PSMS_EINVAL
    assert not out.value


def test_every_tuning_key_is_documented_and_accepted_by_the_library():
    """The binding's tuning keys are the library's: each is named in the header's
    description of psms_set_tuning, and each is a string the library itself holds."""
    from paper_1204_1306_amd import psms

    header = open(HEADER).read()
    for key in psms.Context.TUNING_KEYS:
        assert f'"{key}"' in header, key
    if os.path.exists(psms.LIB_PATH):
        blob = open(psms.LIB_PATH, "rb").read()
        for key in psms.Context.TUNING_KEYS:
            assert key.encode() + b"\0" in blob, key


def test_log_ratio_estimate_matches_the_oracle():
    """psms_log_ratio_estimate (host code of the library, no GPU) against the oracle's
    ln mean_j exp(-Delta_j), on Deltas of ordinary size and on Deltas whose exponentials
    overflow or underflow FP64; bad input gives PSMS_EINVAL."""
    from oracle import estimator
    from paper_1204_1306_amd import psms

    if not os.path.exists(psms.LIB_PATH):
        pytest.skip("libpsms.so not built")
    rng = np.random.default_rng(77)
    d = rng.normal(0.3, 1.2, size=(5, 16))
    got = psms.log_ratio_estimate(d)
    for p in range(5):
        assert got[p] == pytest.approx(estimator.log_ratio_estimate(d[p]), rel=1e-13, abs=1e-14)
    big = np.array([[-800.0, -799.0, -798.5], [900.0, 901.0, 950.0]])  # e^800 overflows, e^-900 underflows
    got = psms.log_ratio_estimate(big)
    for p in range(2):
        assert np.isfinite(got[p])
        assert got[p] == pytest.approx(estimator.log_ratio_estimate(big[p]), rel=1e-13)
    assert psms.log_ratio_estimate([0.0, 0.0])[0] == 0.0  # Delta = 0 exactly: ln 1
    with pytest.raises(psms.PsmsError):
        psms.log_ratio_estimate([[0.0, np.nan]])
    with pytest.raises(psms.PsmsError):
        psms.log_ratio_estimate(np.zeros((1, 0)))
