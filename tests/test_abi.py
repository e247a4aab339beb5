"""CPU checks of the C interface: the library loads and exports every entry
point that include/ads.h declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ads.h")
LIB = os.path.join(ROOT, "paper_2201_02250_amd", "libads.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|int64_t|const char\*)\s+(ads_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["ads_setup", "ads_setup_batched", "ads_apply", "ads_solve", "ads_get_info",
              "ads_export_maps", "ads_partition_bfs", "ads_destroy", "ads_status_string",
              "ads_last_error"]:
        assert s in syms


@pytest.mark.skipif(not os.path.exists(LIB), reason="libads.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s), s
    from paper_2201_02250_amd import ads
    assert sorted(ads.SYMBOLS) == declared_symbols()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libads.so not built")
def test_status_strings_and_null_arguments():
    """Host-side error paths only (no device work): bad arguments are rejected
    with a status code and a message, never an abort."""
    from paper_2201_02250_amd import ads
    L = ads.lib()
    assert ads.ads_status_string(0) == "ADS_OK"
    assert ads.ads_status_string(-4) == "ADS_ERR_SINGULAR"
    out = ctypes.c_void_p()
    assert L.ads_setup(None, None, 0, None, None, ctypes.byref(out)) == ads.ADS_ERR_ARG
    assert "null" in ads.ads_last_error()
    assert L.ads_destroy(None) == 0
    assert L.ads_apply(None, None, None, 1, None) == ads.ADS_ERR_ARG
    assert L.ads_get_info(None, None) == ads.ADS_ERR_ARG
