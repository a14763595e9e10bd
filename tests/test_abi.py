"""The C-ABI library loads and exports every entry point declared in include/mlk.h
(no GPU needed: nothing here calls into the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlk.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mlk_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["mlk_create", "mlk_destroy", "mlk_set_eps", "mlk_add_tls", "mlk_add_multilevel",
                 "mlk_add_plane_source", "mlk_add_point_source", "mlk_add_probe",
                 "mlk_add_flux_plane", "mlk_record_populations", "mlk_step", "mlk_get_field",
                 "mlk_get_series", "mlk_checkpoint_save", "mlk_checkpoint_load"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2512_06173_amd import mlk
    if not os.path.exists(mlk.LIB_PATH):
        pytest.fail("libmlk.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(mlk.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(mlk.exported_symbols()) <= set(_declared())


def test_binding_refuses_to_run_without_the_library(monkeypatch, tmp_path):
    from paper_2512_06173_amd import mlk
    monkeypatch.setattr(mlk, "_lib", None)
    monkeypatch.setattr(mlk, "LIB_PATH", str(tmp_path / "libmlk.so"))
    with pytest.raises(ImportError):
        mlk.lib()
