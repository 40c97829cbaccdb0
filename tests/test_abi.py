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


@pytest.mark.parametrize("n", [8, 16])
def test_library_exports_every_declared_symbol(n):
    path = hydro.lib_path(n)
    if not os.path.exists(path):
        pytest.skip(f"{path} not built (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert sorted(hydro.EXPORTS) == sorted(declared_functions())


@pytest.mark.parametrize("n", [8, 16])
def test_size_helpers_without_gpu(n):
    if not os.path.exists(hydro.lib_path(n)):
        pytest.skip("library not built")
    L = hydro.lib(n)
    assert L.hydro_subgrid_n() == n
    for ns in (0, 5):
        nf = 6 + ns
        assert hydro.q_elems(ns, n) == 26 * nf * (n + 2) ** 3
        assert hydro.f_elems(ns, n) == 3 * nf * (n + 1) * n * n
    assert L.hydro_workspace_bytes() == 0
    assert L.hydro_strerror(-1) == b"invalid argument"


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(hydro, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hydro, "_libs", {})
    with pytest.raises(hydro.HydroError):
        hydro.lib()
    with pytest.raises(hydro.HydroError):
        hydro.lib(12)


def test_copy_blocks_checks_its_arguments_before_the_device():
    if not os.path.exists(hydro.lib_path(8)):
        pytest.skip("library not built")
    L = hydro.lib()
    p = ctypes.c_void_p(16)      # never dereferenced: every call below returns first
    assert L.hydro_copy_blocks(p, 4, p, p, 4, p, None, -1, 8, None) == -1
    assert L.hydro_copy_blocks(p, 4, p, p, 4, p, None, 1, 0, None) == -1
    assert L.hydro_copy_blocks(p, -1, p, p, 4, p, None, 1, 8, None) == -1
    assert L.hydro_copy_blocks(None, 4, p, p, 4, p, None, 1, 8, None) == -1
    assert L.hydro_copy_blocks(p, 4, p, p, 4, None, None, 1, 8, None) == -1
    assert L.hydro_copy_blocks(p, 4, p, p, 4, p, None, 2 ** 30, 2 ** 20, None) == -1
    assert L.hydro_copy_blocks(None, 0, None, None, 0, None, None, 0, 8, None) == 0
