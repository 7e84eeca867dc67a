"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Unit counts must match bit-exactly; float32 results
within the stated tolerances of the float64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

F32_RTOL = 1e-4  # max relative error against the float64 oracle


@pytest.fixture(scope="module")
def d8m():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1608_04431_amd as m
    m._lib.load()  # raises if the HIP library is not built
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_acyclic_dirs(rows, cols, seed, nodata_frac=0.1, noflow_frac=0.02):
    rng = np.random.default_rng(seed)
    z = rng.permutation(rows * cols).astype(np.float32).reshape(rows, cols)
    z[rng.random((rows, cols)) < nodata_frac] = -9999.0
    d = oracle.d8(z)
    d[(rng.random((rows, cols)) < noflow_frac) & (d != 9)] = 8
    return d


def gpu_u32(m, d, tile=(0, 0)):
    out = m.flow_accum(dev(d), acc_type="u32", tile=tile)
    return out.cpu().numpy().view(np.uint32)


def assert_u32_exact(got, d):
    want = oracle.accum_u64(d)
    assert want.max() < 2**32
    np.testing.assert_array_equal(got.astype(np.uint64), want)


def assert_rel(got, want, valid, rtol=F32_RTOL, what=""):
    got = got.astype(np.float64)
    pos = valid & (want > 0)
    rel = np.abs(got[pos] - want[pos]) / want[pos]
    assert rel.size == 0 or rel.max() <= rtol, f"{what} max rel err {rel.max():.3e}"
    zero = valid & (want == 0)
    assert (got[zero] == 0).all(), what
    assert (got[~valid] == 0).all(), what


def assert_adjoint(got, want, valid, what=""):
    """Normwise bound, plus per-cell relative where |lambda| is not tiny."""
    got = got.astype(np.float64)
    scale = np.abs(want[valid]).max() if valid.any() else 0.0
    if scale == 0:
        assert (got == 0).all()
        return
    assert np.abs(got - want)[valid].max() <= F32_RTOL * scale, what
    big = valid & (np.abs(want) >= 1e-3 * scale)
    rel = np.abs(got[big] - want[big]) / np.abs(want[big])
    assert rel.max() <= F32_RTOL, f"{what} max rel err {rel.max():.3e}"
    assert (got[~valid] == 0).all()


# ----------------------------------------------------------------- D8 -------
def test_d8_directions_match_oracle(d8m):
    rng = np.random.default_rng(1)
    cases = [synth.workload_dem("dem512"),
             rng.integers(0, 4, (37, 61)).astype(np.float32),          # many exact ties
             (rng.random((1, 100)) * 5).astype(np.float32),
             (rng.random((100, 1)) * 5).astype(np.float32),
             synth.dem(300, 257, seed=7, lambda0=64, ocean=True)]
    z = cases[1]
    z[rng.random(z.shape) < 0.1] = -9999.0
    z[3, 3] = np.nan
    for z in cases:
        got = d8m.d8_directions(dev(z)).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.d8(z))


def test_d8_directions_strips_blocks_and_alignment(d8m):
    """Shapes that cross the kernel's 64-row strips and 1024-column blocks,
    with and without 4-aligned rows, ties, NoData, NaN and infinities; then the
    same inputs through misaligned input and output pointers (the per-element
    path)."""
    rng = np.random.default_rng(5)
    for shape in [(130, 2052), (129, 2051), (65, 1024), (64, 1025), (3, 4), (200, 8), (1, 1)]:
        z = rng.integers(0, 6, shape).astype(np.float32)
        z[rng.random(shape) < 0.05] = -9999.0
        z[rng.random(shape) < 0.02] = np.nan
        z[rng.random(shape) < 0.01] = np.inf
        z[rng.random(shape) < 0.01] = -np.inf
        want = oracle.d8(z)
        np.testing.assert_array_equal(d8m.d8_directions(dev(z)).cpu().numpy(), want)
        flat = torch.empty(z.size + 1, dtype=torch.float32, device="cuda")
        flat[1:] = dev(z).flatten()
        obuf = torch.zeros(z.size + 3, dtype=torch.uint8, device="cuda")
        out = obuf[1:1 + z.size].view(shape)
        d8m.d8_directions(flat[1:].view(shape), out=out)
        np.testing.assert_array_equal(out.cpu().numpy(), want)
        assert int(obuf[0]) == 0 and (obuf[1 + z.size:] == 0).all()


def test_d8_directions_extreme_magnitudes_and_strip_ends(d8m):
    """Drops whose float products underflow (subnormal and tiny elevations) or
    come near the largest float, where the float slope compare must defer to
    the exact one; and strips whose last row falls on every position of the
    kernel's 6-row unrolled loop (heights 64 + 1 .. 64 + 6 and 6 k), both
    16-byte aligned rows and per-element rows."""
    rng = np.random.default_rng(17)
    scales = [np.float32(2.0 ** -140), np.float32(1e-38), np.float32(2.0 ** -100),
              np.float32(1e38), np.float32(3.0e38)]
    for k, scale in enumerate(scales):
        for shape in [(67, 260), (70, 131)]:
            with np.errstate(over="ignore"):  # 3 x 3e38 becomes +-inf, on purpose
                z = (rng.integers(-3, 4, shape) * scale).astype(np.float32)
            z[rng.random(shape) < 0.03] = -9999.0
            if k >= 3:
                z[rng.random(shape) < 0.02] = np.float32(-3.4e38)
            np.testing.assert_array_equal(d8m.d8_directions(dev(z)).cpu().numpy(), oracle.d8(z),
                                          err_msg=f"scale {scale} shape {shape}")
    for rows in [65, 66, 67, 68, 69, 70, 6, 12, 126, 127]:
        for cols in (256, 257):
            z = synth.dem(rows, cols, seed=rows, lambda0=16, ocean=True)
            np.testing.assert_array_equal(d8m.d8_directions(dev(z)).cpu().numpy(), oracle.d8(z),
                                          err_msg=f"{rows}x{cols}")


def test_d8_directions_near_sqrt2(d8m):
    """The slope compare where the diagonal drop is within a few ulps of
    sqrt(2) times the cardinal one (the kernel's float fast path must defer
    to the exact compare there), per element and 4-aligned."""
    z = synth.sqrt2_blocks()
    np.testing.assert_array_equal(d8m.d8_directions(dev(z)).cpu().numpy(), oracle.d8(z))
    zp = np.concatenate([z, np.full((3, 3), np.float32(1e30), np.float32)], axis=1)
    assert zp.shape[1] % 4 == 0
    np.testing.assert_array_equal(d8m.d8_directions(dev(zp)).cpu().numpy(), oracle.d8(zp))


def test_rho8_directions_match_oracle(d8m):
    """rho8 (random diagonal distance 2 - r per cell) against the oracle on
    terrain with NoData, integer DEMs with ties, strips / blocks / ragged
    edges, the r > 1/2 blocks; and accumulation over rho8 directions."""
    rng = np.random.default_rng(21)
    zi = rng.integers(0, 5, (70, 1030)).astype(np.float32)
    zi[rng.random(zi.shape) < 0.05] = -9999.0
    cases = [synth.dem(300, 257, seed=7, lambda0=64, ocean=True), zi, zi[:, :1029],
             synth.workload_dem("dem512")]
    for i, z in enumerate(cases):
        rnd = synth.uniform(z.shape, 40 + i)
        got = d8m.d8_directions_rho8(dev(z), dev(rnd)).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.rho8(z, rnd), err_msg=f"case {i}")
    rv = synth.uniform((1, 500), 9)[0]
    z, r = synth.rho8_half_blocks(rv)
    zp = np.concatenate([z, np.full((3, 2), np.float32(1e30), np.float32)], axis=1)
    rp = np.concatenate([r, np.full((3, 2), np.float32(0.5), np.float32)], axis=1)
    assert z.shape[1] % 4 == 0 and zp.shape[1] % 4 != 0  # 16-byte and per-element paths
    for zz, rr in ((z, r), (zp, rp)):
        got = d8m.d8_directions_rho8(dev(zz), dev(rr)).cpu().numpy()
        np.testing.assert_array_equal(got, oracle.rho8(zz, rr))
    d = d8m.d8_directions_rho8(dev(cases[3]), dev(synth.uniform(cases[3].shape, 43)))
    assert_u32_exact(d8m.flow_accum(d, acc_type="u32", tile=(64, 48)).cpu().numpy().view(np.uint32),
                     d.cpu().numpy())


# ------------------------------------------------------------ hand fixtures --
def test_golden_fixtures_u32(d8m):
    from conftest import GOLDEN_FILES, load_golden
    for name in GOLDEN_FILES:
        d, A_hand, tile = load_golden(name)
        for t in [tile or (0, 0), (1, 1), (2, 2), (1, 3), (0, 0)]:
            got = gpu_u32(d8m, d, t)
            np.testing.assert_array_equal(got.astype(np.uint64), A_hand, err_msg=f"{name} {t}")


# ------------------------------------------------------- forward, unit counts
@pytest.mark.parametrize("shape,tile", [
    ((1, 1), (0, 0)), ((1, 300), (1, 64)), ((300, 1), (64, 1)), ((1, 300), (0, 0)),
    ((64, 64), (64, 64)), ((65, 63), (64, 64)), ((200, 150), (16, 16)), ((200, 150), (1, 1)),
    ((129, 257), (7, 9)), ((128, 512), (64, 64)), ((300, 200), (32, 48)),
    ((257, 300), (16, 64)),
])
def test_forward_u32_random(d8m, shape, tile):
    d = random_acyclic_dirs(*shape, seed=hash((shape, tile)) % 1000)
    assert_u32_exact(gpu_u32(d8m, d, tile), d)


def test_tile_passes_unaligned_code_rows(d8m):
    """The tile passes read a row of codes that does not start on a 4-byte
    boundary as the aligned words that cover it: widths that are not a
    multiple of four (rows start at every byte offset), and the same rasters
    through code pointers 1, 2 and 3 bytes past an aligned address.  Unit
    counts exact against the oracle, the adjoint within the float32
    tolerance, and the float32 forward and the adjoint equal bit for bit to
    the aligned call."""
    for shape, seed in (((70, 131), 31), ((67, 256), 32), ((45, 97), 33), ((130, 45), 34)):
        d = random_acyclic_dirs(*shape, seed=seed)
        g = dev(synth.uniform(shape, seed + 100))
        want_a = oracle.transpose_f64(d, g.cpu().numpy())
        for tile in ((64, 32), (64, 44), (64, 64), (16, 40)):
            ref_f = d8m.flow_accum(dev(d), g, acc_type="f32", tile=tile)
            ref_a = d8m.flow_accum_adjoint(dev(d), g, tile=tile)
            for off in (0, 1, 2, 3):
                flat = torch.full((d.size + 8,), 0xEE, dtype=torch.uint8, device="cuda")
                flat[off:off + d.size] = dev(d).flatten()
                dv = flat[off:off + d.size].view(shape)
                assert dv.data_ptr() % 4 == off % 4
                what = f"{shape} {tile} +{off}"
                got = d8m.flow_accum(dv, acc_type="u32", tile=tile).cpu().numpy().view(np.uint32)
                assert_u32_exact(got, d)
                assert torch.equal(d8m.flow_accum(dv, g, acc_type="f32", tile=tile), ref_f), what
                lam = d8m.flow_accum_adjoint(dv, g, tile=tile)
                assert torch.equal(lam, ref_a), what
                assert_rel(lam.cpu().numpy(), want_a, d != 9, what=what)


def test_forward_all_nodata_and_outlets(d8m):
    d = np.full((50, 70), 9, dtype=np.uint8)
    assert (gpu_u32(d8m, d) == 0).all()
    d = np.full((50, 70), 8, dtype=np.uint8)          # all NoFlow: every cell 1
    assert (gpu_u32(d8m, d, (16, 16)) == 1).all()
    d = np.full((40, 40), 4, dtype=np.uint8)          # all east, off the raster
    assert_u32_exact(gpu_u32(d8m, d, (8, 8)), d)
    d = np.full((40, 40), 7, dtype=np.uint8)          # diagonal flow across corners
    assert_u32_exact(gpu_u32(d8m, d, (8, 8)), d)
    d = np.full((40, 40), 0, dtype=np.uint8)
    assert_u32_exact(gpu_u32(d8m, d, (5, 3)), d)


def test_tiling_invariance_terrain(d8m):
    z = synth.dem(700, 650, seed=11, lambda0=128, ocean=True)
    d = oracle.d8(z)
    want = oracle.accum_u64(d)
    for tile in [(0, 0), (16, 16), (32, 64), (64, 32), (64, 48), (48, 64), (50, 37), (8, 60), (1, 64), (64, 1)]:
        np.testing.assert_array_equal(gpu_u32(d8m, d, tile).astype(np.uint64), want,
                                      err_msg=str(tile))


def test_dem512_unit_counts(d8m):
    """512 x 512, noise wavelength 128, unit weights, uint32: bit-exact."""
    z = synth.workload_dem("dem512")
    d = oracle.d8(z)
    np.testing.assert_array_equal(d8m.d8_directions(dev(z)).cpu().numpy(), d)
    assert_u32_exact(gpu_u32(d8m, d), d)


# ------------------------------------------------------------ forward, f32 --
@pytest.mark.parametrize("shape,tile", [((200, 150), (16, 16)), ((513, 300), (0, 0)),
                                        ((1, 500), (1, 64)), ((300, 300), (64, 64))])
def test_forward_f32_random(d8m, shape, tile):
    d = random_acyclic_dirs(*shape, seed=7)
    w = synth.uniform(shape, 8)
    got = d8m.flow_accum(dev(d), dev(w), acc_type="f32", tile=tile).cpu().numpy()
    assert_rel(got, oracle.accum_f64(d, w), d != 9, what=str(tile))
    # unit weights through the float path
    got1 = d8m.flow_accum(dev(d), None, acc_type="f32", tile=tile).cpu().numpy()
    assert_rel(got1, oracle.accum_f64(d), d != 9)


def test_forward_f32_deterministic(d8m):
    z = synth.dem(600, 600, seed=12, lambda0=128, ocean=False)
    d = dev(oracle.d8(z))
    w = dev(synth.uniform((600, 600), 13))
    a = d8m.flow_accum(d, w, acc_type="f32")
    for _ in range(3):
        b = d8m.flow_accum(d, w, acc_type="f32")
        assert torch.equal(a, b)


# ---------------------------------------------------------------- adjoint ----
@pytest.mark.parametrize("shape,tile", [((200, 150), (16, 16)), ((513, 300), (0, 0)),
                                        ((1, 500), (1, 64)), ((77, 1), (0, 0)),
                                        ((300, 300), (48, 64)), ((100, 100), (1, 1))])
def test_adjoint_dense(d8m, shape, tile):
    d = random_acyclic_dirs(*shape, seed=21)
    g = synth.uniform(shape, 22)
    got = d8m.flow_accum_adjoint(dev(d), dev(g), tile=tile).cpu().numpy()
    want = oracle.transpose_f64(d, g)
    valid = d != 9
    assert_rel(got, want, valid, what=str(tile))


def test_adjoint_terrain_and_identity(d8m):
    z = synth.dem(640, 700, seed=23, lambda0=128, ocean=True)
    d = oracle.d8(z)
    rng = np.random.default_rng(24)
    w = synth.uniform(d.shape, 25)
    g = np.zeros(d.shape, dtype=np.float32)
    idx = rng.choice(d.size, 64, replace=False)
    g.ravel()[idx] = rng.standard_normal(64).astype(np.float32)
    lam = d8m.flow_accum_adjoint(dev(d), dev(g)).cpu().numpy()
    assert_adjoint(lam, oracle.transpose_f64(d, g), d != 9)
    A = d8m.flow_accum(dev(d), dev(w), acc_type="f32").cpu().numpy().astype(np.float64)
    lhs = float((g.astype(np.float64) * A).sum())
    rhs = float((lam.astype(np.float64) * w).sum())
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), 1.0)


def test_adjoint_unit_cotangent_catchment(d8m):
    z = synth.dem(300, 300, seed=26, lambda0=64, ocean=False)
    d = oracle.d8(z)
    A = oracle.accum_u64(d)
    r, c = np.unravel_index(np.argmax(A), A.shape)
    g = np.zeros(d.shape, dtype=np.float32)
    g[r, c] = 1.0
    lam = d8m.flow_accum_adjoint(dev(d), dev(g), tile=(32, 32)).cpu().numpy()
    assert set(np.unique(lam)) <= {0.0, 1.0}
    assert lam.sum() == A[r, c]


@pytest.mark.parametrize("length", [2186, 2187, 2188, 6562])
def test_long_chain_of_exits(d8m, length):
    """One row flowing east with 1x1 tiles: every cell is a tile and its
    exit, so the exit forest is a single chain of `length` nodes (the flow
    leaves the raster at the east end).  Lengths around powers of three
    check the pointer-jumping round count (each round composes three words)
    and that a complete chain raises no cycle; forward counts are exact, the
    float forward and the adjoint (plain and absorbing) follow the oracle."""
    d = np.full((1, length), 4, dtype=np.uint8)  # code 4 = E
    tile = (1, 1)
    A = d8m.flow_accum(dev(d), acc_type="u32", tile=tile, check=True).cpu().numpy().view(np.uint32)
    np.testing.assert_array_equal(A[0].astype(np.int64), np.arange(1, length + 1))
    w = synth.uniform(d.shape, 41)
    g = synth.uniform(d.shape, 42)
    valid = np.ones(d.shape, bool)
    Af = d8m.flow_accum(dev(d), dev(w), acc_type="f32", tile=tile, check=True).cpu().numpy()
    assert_rel(Af, oracle.accum_f64(d, w), valid, what="f32 forward")
    lam = d8m.flow_accum_adjoint(dev(d), dev(g), tile=tile, check=True).cpu().numpy()
    assert_rel(lam, oracle.transpose_f64(d, g), valid, what="adjoint")
    alpha = np.full(d.shape, 0.999, dtype=np.float32)
    lam_a = d8m.flow_accum_absorb_adjoint(dev(d), dev(alpha), dev(g), tile=tile, check=True).cpu().numpy()
    assert_rel(lam_a, oracle.transpose_absorb_f64(d, alpha, g), valid, what="absorbing adjoint")


# ----------------------------------------------------------------- errors ----
def test_data_errors_reported(d8m):
    d = random_acyclic_dirs(64, 64, 31)
    d[5, 5] = 200
    ws = d8m.Workspace(64, 64)
    d8m.flow_accum(dev(d), ws=ws)
    with pytest.raises(d8m.D8Error) as e:
        d8m.check_status(ws)
    assert e.value.code == -4
    # a two-cell cycle inside one tile, and one across a tile boundary (a
    # cycle of exits, found by forward pass 2 / the adjoint's jumps), for the
    # unit-count, float32 and absorbing forwards and the adjoint
    ones = np.ones((64, 64), np.float32)
    for (r, c), tile in [((10, 10), (0, 0)), ((10, 31), (32, 32))]:
        d = random_acyclic_dirs(64, 64, 32)
        d[r, c], d[r, c + 1] = 4, 3
        ws = d8m.Workspace(64, 64, tile)
        wsa = torch.empty(d8m._lib.load().d8_absorb_workspace_bytes(64, 64, *tile), dtype=torch.uint8,
                          device="cuda")
        for fn, w in ((lambda: d8m.flow_accum(dev(d), ws=ws, tile=tile), ws),
                      (lambda: d8m.flow_accum(dev(d), dev(ones), acc_type="f32", ws=ws, tile=tile), ws),
                      (lambda: d8m.flow_accum_absorb(dev(d), dev(0.5 * ones), dev(ones), tile=tile, ws=wsa), wsa),
                      (lambda: d8m.flow_accum_adjoint(dev(d), dev(ones), ws=ws, tile=tile), ws)):
            fn()
            with pytest.raises(d8m.D8Error) as e:
                d8m.check_status(w)
            assert e.value.code == -5
    # a clean call afterwards resets the status
    d = random_acyclic_dirs(64, 64, 33)
    d8m.flow_accum(dev(d), ws=ws, tile=(32, 32))
    d8m.check_status(ws)


def test_argument_errors(d8m):
    d = dev(random_acyclic_dirs(16, 16, 1))
    with pytest.raises(TypeError):
        d8m.flow_accum(d.float())
    d8m.flow_accum(d, tile=(200, 200))  # clipped to the 16x16 raster: valid
    with pytest.raises(d8m.D8Error):
        d8m.flow_accum(d, tile=(0, 5))
    small = d8m.Workspace(4, 4)
    with pytest.raises(d8m.D8Error) as e:
        d8m.flow_accum(d, ws=small)
    assert e.value.code == -2


def test_empty_raster(d8m):
    d = torch.empty((0, 7), dtype=torch.uint8, device="cuda")
    assert d8m.flow_accum(d).shape == (0, 7)
    g = torch.empty((0, 7), dtype=torch.float32, device="cuda")
    assert d8m.flow_accum_adjoint(d, g).shape == (0, 7)


def test_timing_modes(d8m):
    d = dev(random_acyclic_dirs(200, 150, 4))
    g = dev(synth.uniform((200, 150), 5))
    d8m.timing_report()
    d8m.timing_enable(True)
    d8m.flow_accum(d, tile=(32, 32))
    d8m.flow_accum_adjoint(d, g, tile=(32, 32))
    d8m.timing_enable(False)
    every = d8m.timing_report()
    d8m.timing_enable(True, passes_only=True)
    d8m.flow_accum(d, tile=(32, 32))
    d8m.flow_accum_adjoint(d, g, tile=(32, 32))
    d8m.timing_enable(False)
    passes = d8m.timing_report()
    assert set(passes) == {"fwd_pass1", "fwd_pass2", "adj_pass1", "adj_pass2"}
    assert set(passes) < set(every) and "resolve_fwd" in every
    assert all(n == 1 for _, n in passes.values())
