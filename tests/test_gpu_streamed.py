"""Streamed accumulation of rasters held in host memory (flow_accum_streamed,
flow_accum_streamed_f32, flow_accum_adjoint_streamed): unit counts bit for
bit equal to the oracle and to the in-memory flow_accum with the same tiles,
float sums equal to the in-memory call and within 1e-4 of the oracle, the
adjoint within 1e-4 of the oracle's transpose, over band sizes from one
tile row to the whole raster, ragged edges, NoData / NoFlow, pinned and
pageable host memory, data errors."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def d8m():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1608_04431_amd as m
    m._lib.load()
    return m


def random_acyclic_dirs(rows, cols, seed, nodata_frac=0.1, noflow_frac=0.02):
    rng = np.random.default_rng(seed)
    z = rng.permutation(rows * cols).astype(np.float32).reshape(rows, cols)
    z[rng.random((rows, cols)) < nodata_frac] = -9999.0
    d = oracle.d8(z)
    d[(rng.random((rows, cols)) < noflow_frac) & (d != 9)] = 8
    return d


def streamed(m, d, tile, band, pin=True):
    h = torch.from_numpy(np.ascontiguousarray(d))
    if pin:
        h = h.pin_memory()
    return m.flow_accum_streamed(h, tile=tile, band_rows=band).numpy().view(np.uint32)


@pytest.mark.parametrize("shape,tile,bands", [
    ((300, 257), (32, 32), (32, 64, 96, 0, 1024)),
    ((200, 131), (16, 24), (16, 48, 112)),
    ((97, 64), (8, 64), (8, 40)),
])
def test_streamed_matches_oracle_and_in_memory(d8m, shape, tile, bands):
    cases = [random_acyclic_dirs(*shape, seed=sum(shape)),
             oracle.d8(synth.dem(*shape, seed=11, lambda0=32, ocean=True))]
    for d in cases:
        want = oracle.accum_u64(d)
        ref = d8m.flow_accum(torch.from_numpy(d).cuda(), acc_type="u32", tile=tile)
        ref = ref.cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(ref.astype(np.uint64), want)
        for band in bands:
            got = streamed(d8m, d, tile, band)
            np.testing.assert_array_equal(got, ref, err_msg=f"band_rows {band}")


def test_streamed_terrain_pageable_and_repeated(d8m):
    d = oracle.d8(synth.workload_dem("dem512"))
    ref = d8m.flow_accum(torch.from_numpy(d).cuda(), acc_type="u32", tile=(64, 48))
    ref = ref.cpu().numpy().view(np.uint32)
    ws = torch.empty(d8m.stream_workspace_bytes(512, 512, (64, 48), 64), dtype=torch.uint8,
                     device="cuda")
    h = torch.from_numpy(d)
    for _ in range(2):  # pageable host memory, one workspace reused
        got = d8m.flow_accum_streamed(h, tile=(64, 48), band_rows=64, ws=ws)
        np.testing.assert_array_equal(got.numpy().view(np.uint32), ref)
    np.testing.assert_array_equal(streamed(d8m, d, (64, 48), 128), ref)


def test_streamed_errors_and_empty(d8m):
    with pytest.raises(d8m.D8Error):
        d8m.stream_workspace_bytes(100, 100, (32, 32), 48)     # not whole tile rows
    with pytest.raises(d8m.D8Error):
        d8m.stream_workspace_bytes(100, 100, (32, 32), -32)
    out = d8m.flow_accum_streamed(torch.zeros((0, 7), dtype=torch.uint8), tile=(8, 8))
    assert out.shape == (0, 7)
    d = random_acyclic_dirs(64, 64, 31)
    d[40, 5] = 200
    with pytest.raises(d8m.D8Error) as e:
        streamed(d8m, d, (16, 16), 16)
    assert e.value.code == -4
    d = random_acyclic_dirs(64, 64, 32)
    d[31, 10], d[32, 10] = 6, 1                                  # a cycle across two bands
    with pytest.raises(d8m.D8Error) as e:
        streamed(d8m, d, (16, 16), 32)
    assert e.value.code == -5
    d = random_acyclic_dirs(64, 64, 33)                          # clean again
    got = streamed(d8m, d, (16, 16), 16)
    np.testing.assert_array_equal(got.astype(np.uint64), oracle.accum_u64(d))


def f32_close(got, want, valid, rtol=1e-4):
    got = got.astype(np.float64)
    pos = valid & (want > 0)
    rel = np.abs(got[pos] - want[pos]) / want[pos]
    assert rel.size == 0 or rel.max() <= rtol, rel.max()
    assert (got[valid & (want == 0)] == 0).all() and (got[~valid] == 0).all()


@pytest.mark.parametrize("shape,tile,bands", [
    ((300, 257), (32, 32), (32, 96, 0, 1024)),
    ((200, 131), (16, 24), (16, 48)),
])
def test_streamed_f32_and_adjoint(d8m, shape, tile, bands):
    """Float weights and the adjoint streamed from host memory: the float
    forward equals the in-memory call bit for bit (same tiles, the same
    fixed-order sums) and the oracle within 1e-4 per cell, unit weights too;
    the adjoint (tiles recomputed with the exits seeded) within 1e-4 per cell
    of the oracle's transpose."""
    cases = [random_acyclic_dirs(*shape, seed=sum(shape) + 1),
             oracle.d8(synth.dem(*shape, seed=12, lambda0=32, ocean=True))]
    for d in cases:
        valid = d != 9
        w = synth.uniform(shape, 41)
        g = synth.uniform(shape, 42)
        ref = d8m.flow_accum(torch.from_numpy(d).cuda(), torch.from_numpy(w).cuda(), acc_type="f32",
                             tile=tile).cpu()
        f32_close(ref.numpy(), oracle.accum_f64(d, w), valid)
        want_lam = oracle.transpose_f64(d, g)
        dh = torch.from_numpy(d).pin_memory()
        wh, gh = torch.from_numpy(w).pin_memory(), torch.from_numpy(g).pin_memory()
        for band in bands:
            got = d8m.flow_accum_streamed_f32(dh, wh, tile=tile, band_rows=band)
            assert torch.equal(got, ref), f"band_rows {band}"
            lam = d8m.flow_accum_adjoint_streamed(dh, gh, tile=tile, band_rows=band)
            f32_close(lam.numpy(), want_lam, valid)
        one = d8m.flow_accum_streamed_f32(dh, None, tile=tile, band_rows=bands[0])
        np.testing.assert_array_equal(one.numpy().astype(np.float64), oracle.accum_u64(d).astype(np.float64))


def test_streamed_float_errors(d8m):
    d = random_acyclic_dirs(64, 64, 34)
    d[31, 10], d[32, 10] = 6, 1                                  # a cycle across two bands
    g = torch.from_numpy(synth.uniform((64, 64), 43))
    with pytest.raises(d8m.D8Error) as e:
        d8m.flow_accum_adjoint_streamed(torch.from_numpy(d), g, tile=(16, 16), band_rows=32)
    assert e.value.code == -5
    with pytest.raises(d8m.D8Error) as e:
        d8m.flow_accum_streamed_f32(torch.from_numpy(d), g, tile=(16, 16), band_rows=32)
    assert e.value.code == -5
    ws = torch.empty(d8m.stream_workspace_bytes(64, 64, (16, 16), 32), dtype=torch.uint8, device="cuda")
    lib = d8m._lib.load()
    rc = lib.flow_accum_adjoint_streamed(torch.from_numpy(d).data_ptr(), None, g.data_ptr(), 64, 64, 16, 16,
                                         32, ws.data_ptr(), ws.numel(), None)
    assert rc == d8m._lib.D8_EINVAL                              # the cotangent is required
    out = d8m.flow_accum_adjoint_streamed(torch.zeros((5, 0), dtype=torch.uint8), torch.zeros((5, 0)),
                                          tile=(8, 8))
    assert out.shape == (5, 0)
