"""The C-ABI library loads on the CPU host and exports every function that
include/hydro.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

from paper_2210_06439_amd import hydro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hydro.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("hydro_reconstruct", "hydro_flux", "hydro_divergence", "hydro_step"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(hydro.LIB_PATH):
        pytest.skip("libhydro.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(hydro.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(hydro.EXPORTS) == sorted(declared_functions())


def test_size_helpers_without_gpu():
    if not os.path.exists(hydro.LIB_PATH):
        pytest.skip("libhydro.so not built")
    assert hydro.q_elems(5) == 286000 and hydro.f_elems(5) == 19008
    assert hydro.lib().hydro_workspace_bytes() == 0
    assert hydro.lib().hydro_strerror(-1) == b"invalid argument"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(hydro, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hydro, "_lib", None)
    with pytest.raises(hydro.HydroError):
        hydro.lib()
