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


def test_binding_structs_match_the_header(tmp_path):
    """Every struct the binding mirrors has the header's size and field offsets (a C
    program compiled against include/lfmm.h prints them)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"lfmm_options": lfmm.Options, "lfmm_report": lfmm.Report, "lfmm_tune_report": lfmm.TuneReport,
               "lfmm_train_opts": lfmm.TrainOpts, "lfmm_train_report": lfmm.TrainReport,
               "lfmm_table_opts": lfmm.TableOpts, "lfmm_table_report": lfmm.TableReport}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "lfmm.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for f, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, f, cname, f))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, c = ln.split()
            got[(a, b)] = int(c)
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
