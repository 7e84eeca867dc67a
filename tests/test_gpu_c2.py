"""The 8192 x 8192 workload with ocean discs (dem8192_ocean: >= 10 % NoData in
random circular masks, float32 weights U[0, 1) with seed 21), checked over the
whole raster against the oracle: D8 codes byte for byte, unit counts bit for
bit, float32 weighted accumulation per cell within 1e-4 of the float64
oracle (max relative error over data cells with a positive reference, and
exactly 0 where the reference is 0).  Eq. (1); NoData handling at the entry of
Algorithm 1.  The tile shapes are the autotuner's choice for this size (the
launch the library makes with tile 0 x 0) and a second, fixed shape."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

F32_RTOL = 1e-4


@pytest.fixture(scope="module")
def d8m():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1608_04431_amd as m
    m._lib.load()
    return m


@pytest.fixture(scope="module")
def c2():
    wl = synth.WORKLOADS["dem8192_ocean"]
    z = synth.workload_dem("dem8192_ocean")
    d_ref = oracle.d8(z)
    w = synth.uniform(z.shape, wl["seed_w"])
    return dict(z=z, d=d_ref, w=w, A_u=oracle.accum_u64(d_ref), A_f=oracle.accum_f64(d_ref, w))


def test_c2_inputs_have_ocean(c2):
    nodata = float((c2["d"] == 9).mean())
    assert nodata >= 0.10, nodata
    # NoData must not be one blob: several coasts, cells of every other kind
    assert (c2["d"] == 8).any() and (c2["d"] < 8).mean() > 0.8


def test_c2_d8_whole_raster(d8m, c2):
    got = d8m.d8_directions(torch.from_numpy(c2["z"]).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got, c2["d"])


@pytest.mark.parametrize("tile", [(0, 0), (64, 64)])
def test_c2_unit_counts_bit_exact(d8m, c2, tile):
    d = torch.from_numpy(c2["d"]).cuda()
    got = d8m.flow_accum(d, acc_type="u32", tile=tile).cpu().numpy().view(np.uint32)
    want = c2["A_u"]
    assert want.max() < 2 ** 32
    np.testing.assert_array_equal(got.astype(np.uint64), want)


@pytest.mark.parametrize("tile", [(0, 0), (64, 64)])
def test_c2_weighted_f32_per_cell(d8m, c2, tile):
    d = torch.from_numpy(c2["d"]).cuda()
    w = torch.from_numpy(c2["w"]).cuda()
    got = d8m.flow_accum(d, w, acc_type="f32", tile=tile).cpu().numpy().astype(np.float64)
    want = c2["A_f"]
    valid = c2["d"] != 9
    pos = valid & (want > 0)
    rel = np.abs(got[pos] - want[pos]) / want[pos]
    assert rel.max() <= F32_RTOL, f"max rel err {rel.max():.3e} at tile {tile}"
    assert (got[valid & (want == 0)] == 0).all()
    assert (got[~valid] == 0).all()
    # the unit-weight float path on the same raster equals the exact counts
    # wherever they are below 2^24 (every count is a sum of ones)
    got1 = d8m.flow_accum(d, None, acc_type="f32", tile=tile).cpu().numpy().astype(np.float64)
    small = valid & (c2["A_u"] < 2 ** 24)
    np.testing.assert_array_equal(got1[small], c2["A_u"][small].astype(np.float64))


def test_c2_weighted_f32_repeats_bit_for_bit(d8m, c2):
    """Float32 sums are taken in an order fixed by the input (within tiles by
    the one wavefront's LDS order, across tiles by node id and direction), so
    repeated calls agree bit for bit, on two tile shapes."""
    d = torch.from_numpy(c2["d"]).cuda()
    w = torch.from_numpy(c2["w"]).cuda()
    for tile in ((0, 0), (16, 16)):
        a = d8m.flow_accum(d, w, acc_type="f32", tile=tile)
        for _ in range(3):
            assert torch.equal(a, d8m.flow_accum(d, w, acc_type="f32", tile=tile)), tile
