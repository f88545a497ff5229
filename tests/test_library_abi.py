"""CPU-side checks of the C ABI: the library loads and exports every declared entry point."""
import ctypes
import os

import pytest

from paper_2403_13406_amd import _lib


def test_header_declares_the_expected_calls():
    names = _lib.declared_functions()
    for n in ("eslb_create", "eslb_step", "eslb_init_equilibrium", "eslb_moments", "eslb_relax",
              "eslb_transport", "eslb_gather", "eslb_diagnostics", "eslb_destroy"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="libeslb.so not built")
def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    missing = [n for n in _lib.declared_functions() if not hasattr(lib, n)]
    assert missing == []
    # host-only entry points work without a device
    assert lib.eslb_status_string(-1) == b"invalid argument"
    ctx = ctypes.c_void_p()
    p = _lib.Problem()
    p.lattice, p.system, p.nx, p.ny = 1, 3, 16, 1   # Euler on D1Q2: unsupported, rejected before any HIP call
    p.kappa, p.relax, p.scheme, p.V, p.dx, p.omega = 1, 1, 1, 1.0, 1.0 / 16, 2.0
    p.param[0] = 1.4
    assert lib.eslb_create(ctypes.byref(p), None, ctypes.byref(ctx)) == _lib.ERR_UNSUPPORTED
    assert b"D2Q4" in lib.eslb_last_error(None)
    p.lattice, p.system, p.nx = 2, 3, 0
    assert lib.eslb_create(ctypes.byref(p), None, ctypes.byref(ctx)) == _lib.ERR_INVALID_ARG


def test_product_path_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()
