"""The C-ABI library loads and exports every symbol include/d8flow.h declares;
host-side argument checks (no GPU needed: they return before any launch)."""
import ctypes
import os
import re

import pytest

from paper_1608_04431_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "d8flow.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(d8_\w+|flow_accum\w*)\s*\(", src)))


def test_exports_match_header():
    lib = _lib.load()
    names = header_functions()
    assert set(names) == set(_lib.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n
        assert ctypes.cast(getattr(lib, n), ctypes.c_void_p).value


def test_strerror_and_version():
    lib = _lib.load()
    assert lib.d8_version() >= 100
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.d8_strerror(code)
    assert b"unknown" in lib.d8_strerror(42)


def test_workspace_bytes():
    lib = _lib.load()
    assert lib.d8_workspace_bytes(512, 512, 64, 64) > 0
    assert lib.d8_workspace_bytes(512, 512, 0, 0) == lib.d8_workspace_bytes(512, 512, 64, 64)
    assert lib.d8_workspace_bytes(512, 512, 200, 200) == 0        # > 8192 cells per tile
    assert lib.d8_workspace_bytes(10, 10, 200, 200) > 0           # clipped to the raster
    assert lib.d8_workspace_bytes(512, 512, 0, 5) == 0
    assert lib.d8_workspace_bytes(-1, 5, 8, 8) == 0
    assert lib.d8_workspace_bytes(0, 5, 8, 8) > 0                 # empty raster: status only
    # grows with the perimeter count: smaller tiles need more
    assert lib.d8_workspace_bytes(1024, 1024, 16, 16) > lib.d8_workspace_bytes(1024, 1024, 64, 64)


def test_argument_errors_return_before_launch():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)
    # bad acc type / weights with u32 / bad tile / negative size
    assert lib.flow_accum(fake, None, fake, 7, 4, 4, 0, 0, fake, 1 << 20, None) == _lib.D8_EINVAL
    assert lib.flow_accum(fake, fake, fake, _lib.D8_ACC_U32, 4, 4, 0, 0, fake, 1 << 20,
                          None) == _lib.D8_EINVAL
    assert lib.flow_accum(fake, None, fake, 0, 4, 4, 0, 3, fake, 1 << 20, None) == _lib.D8_EINVAL
    assert lib.flow_accum(fake, None, fake, 0, -4, 4, 0, 0, fake, 1 << 20, None) == _lib.D8_EINVAL
    # missing / small workspace
    assert lib.flow_accum(fake, None, fake, 0, 4, 4, 0, 0, None, 0, None) == _lib.D8_EWORKSPACE
    assert lib.flow_accum(fake, None, fake, 0, 64, 64, 0, 0, fake, 100, None) == _lib.D8_EWORKSPACE
    assert lib.flow_accum_adjoint(fake, fake, fake, 64, 64, 0, 0, fake, 100,
                                  None) == _lib.D8_EWORKSPACE
    # null arrays
    assert lib.flow_accum(None, None, fake, 0, 4, 4, 0, 0, fake, 1 << 20, None) == _lib.D8_EINVAL
    assert lib.flow_accum_adjoint(fake, None, fake, 4, 4, 0, 0, fake, 1 << 20,
                                  None) == _lib.D8_EINVAL
    assert lib.d8_directions(None, fake, 4, 4, 0.0, None) == _lib.D8_EINVAL
    assert lib.d8_directions(fake, fake, -1, 4, 0.0, None) == _lib.D8_EINVAL
    assert lib.d8_check_status(None, None) == _lib.D8_EINVAL
    # empty raster, no workspace needed for d8_directions
    assert lib.d8_directions(None, None, 0, 4, 0.0, None) == _lib.D8_OK


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()
