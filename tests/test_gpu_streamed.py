"""Streamed accumulation of rasters held in host memory (flow_accum_streamed):
bit for bit equal to the oracle and to the in-memory flow_accum with the same
tiles, over band sizes from one tile row to the whole raster, ragged edges,
NoData / NoFlow, pinned and pageable host memory, data errors."""
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
