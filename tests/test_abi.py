"""The C-ABI library loads and exports every entry point its header declares
(no compute calls: this runs without a GPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpnl.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mpnl_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mpnl_create", "mpnl_destroy", "mpnl_detect", "mpnl_slot_prepare",
                 "mpnl_slot_detect", "mpnl_slot_release", "mpnl_detect_batch", "mpnl_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2409_14355_amd as mp
    lib = mp.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(mp.EXPORTED)
    nm = subprocess.run(["nm", "-D", "--defined-only", mp.LIB_PATH], capture_output=True, text=True)
    exported = set(re.findall(r"\bT (mpnl_\w+)", nm.stdout))
    assert set(declared_functions()) <= exported


def test_strerror_needs_no_gpu():
    import paper_2409_14355_amd as mp
    assert "invalid" in mp.strerror(mp.MPNL_E_INVAL)
    assert "budget" in mp.strerror(mp.MPNL_E_NOMEM)
    assert mp.strerror(12345) == "unknown error code"


def test_no_cpu_fallback_in_the_package():
    """The product path never reaches the oracle."""
    pkg = os.path.join(ROOT, "paper_2409_14355_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".inc", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle-", ""), f
