"""CPU checks of the C ABI: the built library loads and exports every symbol the
public header declares (no compute call is made without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2106_12487_amd import blochwave

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_paper_calls():
    names = blochwave.header_symbols()
    for required in ("bw_create_rve", "bw_destroy_rve", "bw_apply_K", "bw_apply_M", "bw_pcg_solve",
                     "bw_lowest_modes", "bw_last_error"):
        assert required in names


def test_library_exports_every_header_symbol():
    if not os.path.exists(blochwave.LIB_PATH):
        pytest.fail("libblochwave.so is not built (run python -m paper_2106_12487_amd.build_lib)")
    L = ctypes.CDLL(blochwave.LIB_PATH)
    missing = [n for n in blochwave.header_symbols() if not hasattr(L, n)]
    assert not missing, missing
    # every header function has a ctypes signature in the binding
    assert set(blochwave.header_symbols()) <= set(blochwave._SIGS)


def test_header_is_plain_c():
    txt = open(os.path.join(ROOT, "include", "blochwave.h")).read()
    assert 'extern "C"' in txt
    assert not re.search(r"\btorch\b|\bat::|std::", txt)
