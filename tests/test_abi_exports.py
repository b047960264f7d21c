"""The C-ABI library loads and exports every function include/nepspin.h declares
(no compute call: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nepspin.h")
LIB = os.path.join(ROOT, "paper_2606_14073_amd", "libnepspin.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", src, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("nep_spin_eval", "sl_integrate_steps", "sl_replica_submit", "sl_replica_poll"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(lib, n), n
    from paper_2606_14073_amd import nepspin
    assert sorted(nepspin.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_error_reporting_without_device_work():
    from paper_2606_14073_amd import nepspin
    L = nepspin.load()
    # NULL arguments are rejected before any device call
    assert L.nep_model_create(None, None, 0, None) == nepspin.SL_E_INVALID
    assert b"NULL" in L.sl_last_error() or len(L.sl_last_error()) > 0
    assert L.sl_integrate_steps(None, 1, None) == nepspin.SL_E_INVALID
    assert L.sl_replica_poll(None, 1, None) == nepspin.SL_E_INVALID
