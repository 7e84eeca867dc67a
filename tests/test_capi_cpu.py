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
    assert lib.d8_timing_enable(3) == _lib.D8_EINVAL
    assert lib.d8_timing_enable(-1) == _lib.D8_EINVAL
    assert lib.d8_timing_enable(0) == _lib.D8_OK


def test_workspace_bytes():
    lib = _lib.load()
    assert lib.d8_workspace_bytes(512, 512, 64, 64) > 0
    assert lib.d8_workspace_bytes(512, 512, 0, 0) == lib.d8_workspace_bytes(512, 512, 64, 64)
    assert lib.d8_workspace_bytes(512, 512, 200, 200) == 0        # a side above 64
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
    # missing / misaligned / small workspace
    odd = ctypes.c_void_p(0x1000 + 16)
    assert lib.flow_accum(fake, None, fake, 0, 4, 4, 0, 0, odd, 1 << 20, None) == _lib.D8_EWORKSPACE
    assert lib.flow_accum_adjoint(fake, fake, fake, 4, 4, 0, 0, odd, 1 << 20,
                                  None) == _lib.D8_EWORKSPACE
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


def test_stream_workspace_and_argument_errors():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)
    n = lib.d8_stream_workspace_bytes(1000, 300, 64, 48, 128)
    assert n > lib.d8_workspace_bytes(1000, 300, 64, 48) // 2
    assert lib.d8_stream_workspace_bytes(1000, 300, 64, 48, 0) > 0          # default bands
    assert lib.d8_stream_workspace_bytes(1000, 300, 64, 48, 100) == 0       # not whole tile rows
    assert lib.d8_stream_workspace_bytes(1000, 300, 64, 48, -64) == 0
    assert lib.d8_stream_workspace_bytes(0, 300, 64, 48, 64) > 0            # empty: status only
    # bigger bands need bigger slots; bands beyond the raster are cut to it
    assert lib.d8_stream_workspace_bytes(1000, 300, 64, 48, 256) > n
    assert lib.d8_stream_workspace_bytes(1000, 300, 64, 48, 4096) == \
        lib.d8_stream_workspace_bytes(1000, 300, 64, 48, 1024)
    EINVAL, EWS = _lib.D8_EINVAL, _lib.D8_EWORKSPACE
    assert lib.flow_accum_streamed(fake, fake, 1000, 300, 64, 48, 100, fake, n, None) == EINVAL
    assert lib.flow_accum_streamed(None, fake, 1000, 300, 64, 48, 128, fake, n, None) == EINVAL
    assert lib.flow_accum_streamed(fake, fake, 1000, 300, 64, 48, 128, fake, n - 1, None) == EWS
    assert lib.flow_accum_streamed(fake, fake, 1000, 300, 64, 48, 128, None, n, None) == EWS
    odd = ctypes.c_void_p(0x1000 + 8)
    assert lib.flow_accum_streamed(fake, fake, 1000, 300, 64, 48, 128, odd, n, None) == EWS


def test_absorb_workspace_and_argument_errors():
    lib = _lib.load()
    fake = ctypes.c_void_p(0x1000)
    n = lib.d8_absorb_workspace_bytes(1000, 300, 64, 48)
    assert n > lib.d8_workspace_bytes(1000, 300, 64, 48)      # alpha path products per node
    assert lib.d8_absorb_workspace_bytes(1000, 300, 64, -1) == 0
    assert lib.d8_absorb_workspace_bytes(0, 300, 64, 48) == 512
    EINVAL, EWS = _lib.D8_EINVAL, _lib.D8_EWORKSPACE
    assert lib.flow_accum_absorb(fake, None, None, fake, 1000, 300, 64, 48, fake, n, None) == EINVAL
    assert lib.flow_accum_absorb(None, None, fake, fake, 1000, 300, 64, 48, fake, n, None) == EINVAL
    assert lib.flow_accum_absorb(fake, None, fake, fake, 1000, 300, 64, -1, fake, n, None) == EINVAL
    assert lib.flow_accum_absorb(fake, None, fake, fake, 1000, 300, 64, 48, fake, n - 1, None) == EWS
    odd = ctypes.c_void_p(0x1000 + 8)
    assert lib.flow_accum_absorb(fake, None, fake, fake, 1000, 300, 64, 48, odd, n, None) == EWS
    adj = lib.flow_accum_absorb_adjoint
    assert adj(fake, None, fake, fake, 1000, 300, 64, 48, fake, n, None) == EINVAL      # no alpha
    assert adj(fake, fake, None, fake, 1000, 300, 64, 48, fake, n, None) == EINVAL      # no g
    assert adj(fake, fake, fake, None, 1000, 300, 64, 48, fake, n, None) == EINVAL      # no out
    assert adj(fake, fake, fake, fake, 1000, 300, 64, -1, fake, n, None) == EINVAL
    assert adj(fake, fake, fake, fake, 1000, 300, 64, 48, fake, n - 1, None) == EWS
    assert adj(fake, fake, fake, fake, 1000, 300, 64, 48, odd, n, None) == EWS
    ag = lib.flow_accum_absorb_alpha_grad
    assert ag(None, fake, fake, fake, 10, 10, None) == EINVAL
    assert ag(fake, fake, None, fake, 10, 10, None) == EINVAL
    assert ag(fake, fake, fake, fake, -1, 10, None) == EINVAL
    assert ag(None, None, None, None, 0, 10, None) == _lib.D8_OK      # empty: nothing to do


def test_batch_argument_errors_return_before_launch():
    lib = _lib.load()
    fake = 0x1000
    It = _lib.BatchItem
    items = (It * 3)(It(fake, None, fake, None, None, 100, 80, 0, 0),
                     It(fake, None, fake, fake, fake, 0, 50, 0, 0),     # empty: skipped
                     It(fake, fake, fake, None, None, 300, 20, 32, 16))
    nb = lib.d8_batch_workspace_bytes(items, 3)
    assert nb > lib.d8_batch_workspace_bytes(items, 1) > lib.d8_batch_workspace_bytes(items, 0) > 0
    bad = (It * 1)(It(fake, None, fake, None, None, -1, 8, 0, 0))
    assert lib.d8_batch_workspace_bytes(bad, 1) == 0
    bad = (It * 1)(It(fake, None, fake, None, None, 100, 100, 0, 5))
    assert lib.d8_batch_workspace_bytes(bad, 1) == 0
    bad = (It * 1)(It(None, None, fake, None, None, 10, 10, 0, 0))   # no directions
    assert lib.d8_batch_workspace_bytes(bad, 1) == 0
    EINVAL, EWS = _lib.D8_EINVAL, _lib.D8_EWORKSPACE
    FWD, ADJ = _lib.D8_BATCH_FWD, _lib.D8_BATCH_ADJ
    assert lib.flow_accum_batched(items, 3, 0, fake, nb, None) == EINVAL
    assert lib.flow_accum_batched(items, 3, 4, fake, nb, None) == EINVAL
    assert lib.flow_accum_batched(items, 3, ADJ, fake, nb, None) == EINVAL   # item 0 has no g
    assert lib.flow_accum_batched(items, 3, FWD, fake, nb - 1, None) == EWS
    assert lib.flow_accum_batched(items, 3, FWD, None, 0, None) == EWS
    assert lib.flow_accum_batched(items, 3, FWD, fake + 64, nb + 64, None) == EWS  # misaligned
    assert lib.flow_accum_batched(None, 3, FWD, fake, nb, None) == EINVAL
    assert lib.flow_accum_batched(items, -1, FWD, fake, nb, None) == EINVAL
    h = ctypes.c_void_p()
    assert lib.d8_graph_create(items, 3, 0, fake, nb, None, ctypes.byref(h)) == EINVAL
    assert h.value is None
    assert lib.d8_graph_create(items, 3, FWD, fake, nb, None, None) == EINVAL
    assert lib.d8_graph_launch(None, None) == EINVAL
    assert lib.d8_graph_destroy(None) == EINVAL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        _lib.load()


def _nnodes(rows, cols, th, tw):
    """Perimeter cells of all tiles (every tile's ring, edge tiles smaller)."""
    def ring(h, w):
        return h * w if h <= 2 or w <= 2 else 2 * (h + w) - 4
    n = 0
    for r0 in range(0, rows, th):
        for c0 in range(0, cols, tw):
            n += ring(min(th, rows - r0), min(tw, cols - c0))
    return n


@pytest.mark.parametrize("rows,cols,th,tw,band", [(32768, 32768, 64, 44, 1024), (4096, 4096, 16, 16, 64),
                                                   (3000, 2000, 8, 8, 8)])
def test_workspaces_hold_the_float_resolve_lists(rows, cols, th, tw, band):
    """Every workspace the float forward can run in holds its per-node arrays
    (link 2, entry/succ/indeg/counts/A_loc 4 each, two 8-byte words) and the
    resolve's children lists (three words per node) that lie over the
    adjoint's labels or the streamed slots."""
    lib = _lib.load()
    N = _nnodes(rows, cols, th, tw)
    need = 512 + N * (2 + 5 * 4 + 2 * 8) + 3 * N * 4
    assert lib.d8_workspace_bytes(rows, cols, th, tw) >= need
    assert lib.d8_stream_workspace_bytes(rows, cols, th, tw, band) >= need
    assert lib.d8_absorb_workspace_bytes(rows, cols, th, tw) >= need
