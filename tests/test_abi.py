"""CPU-side checks of the C-ABI library: it loads and exports every symbol declared
in include/psms.h, and argument errors are reported without touching a GPU."""
import ctypes
import os
import re

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
