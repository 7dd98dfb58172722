"""Host-side checks of the HIP library: it loads and exports every declared symbol."""
import ctypes
import os

import pytest

from paper_1902_05132_amd import lfmm


def test_header_declares_the_boundary():
    names = lfmm.exported_symbols_from_header()
    for required in ("lfmm_plan", "lfmm_eval", "lfmm_eval_device", "lfmm_destroy", "lfmm_last_report",
                     "lfmm_translation", "lfmm_reaction_operator", "lfmm_densities"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(lfmm.LIB_PATH), reason="liblfmm.so not built")
def test_library_loads_and_exports_every_declared_symbol():
    lib = ctypes.CDLL(lfmm.LIB_PATH)
    for name in lfmm.exported_symbols_from_header():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(lfmm.LIB_PATH), reason="liblfmm.so not built")
def test_status_strings():
    lib = lfmm.load()
    assert lib.lfmm_status_string(0) == b"ok"
    assert lib.lfmm_status_string(1) == b"invalid argument"
    assert lib.lfmm_stage_name(0) == b"classify"
    assert lib.lfmm_stage_name(99) is None


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(lfmm, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(lfmm, "_lib", None)
    with pytest.raises(ImportError):
        lfmm.load()
