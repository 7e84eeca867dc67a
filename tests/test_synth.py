"""Pins for the input generator (it is not part of the method, but both sides
of every parity test consume it).  CPU only."""
import numpy as np
import pytest

import oracle
import synth

DR = [-1, -1, -1, 0, 0, 1, 1, 1]
DC = [-1, 0, 1, -1, 1, -1, 0, 1]
NOD = np.iinfo(np.int32).min


def minimax_spill(zi):
    """Brute-force Priority-Flood result for epsilon = 0: the lowest level at
    which each cell can drain to a seed (border cell or NoData neighbour),
    i.e. min over paths of the max elevation on the path, by relaxation."""
    rows, cols = zi.shape
    data = zi != NOD
    seed = np.zeros_like(data)
    for r in range(rows):
        for c in range(cols):
            if not data[r, c]:
                continue
            if r in (0, rows - 1) or c in (0, cols - 1):
                seed[r, c] = True
            for k in range(8):
                rr, cc = r + DR[k], c + DC[k]
                if 0 <= rr < rows and 0 <= cc < cols and not data[rr, cc]:
                    seed[r, c] = True
    f = np.where(seed, zi.astype(np.int64), np.iinfo(np.int64).max)
    changed = True
    while changed:
        changed = False
        for r in range(rows):
            for c in range(cols):
                if not data[r, c] or seed[r, c]:
                    continue
                best = f[r, c]
                for k in range(8):
                    rr, cc = r + DR[k], c + DC[k]
                    if 0 <= rr < rows and 0 <= cc < cols and data[rr, cc]:
                        cand = max(int(zi[r, c]), int(f[rr, cc]))
                        if cand < best:
                            best = cand
                if best < f[r, c]:
                    f[r, c] = best
                    changed = True
    return np.where(data, f, NOD), seed


@pytest.mark.parametrize("seed", range(5))
def test_fill_eps0_equals_minimax_spill(seed):
    rng = np.random.default_rng(seed)
    rows, cols = [(12, 15), (20, 20), (1, 9), (9, 1), (25, 31)][seed]
    zi = rng.integers(0, 30, (rows, cols)).astype(np.int32)
    zi[rng.random(zi.shape) < 0.1] = NOD
    want, _ = minimax_spill(zi)
    got = synth.fill_int(zi.copy(), 0)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("seed", range(3))
def test_fill_eps_invariants(seed):
    rng = np.random.default_rng(10 + seed)
    zi = rng.integers(0, 50, (30, 40)).astype(np.int32)
    zi[rng.random(zi.shape) < 0.08] = NOD
    _, seed_mask = minimax_spill(zi)
    f = synth.fill_int(zi.copy(), 1)
    data = zi != NOD
    assert (f[~data] == NOD).all()
    assert (f[data] >= zi[data]).all()
    rows, cols = zi.shape
    for r in range(rows):
        for c in range(cols):
            if not data[r, c] or seed_mask[r, c]:
                continue
            lower = any(0 <= r + DR[k] < rows and 0 <= c + DC[k] < cols and
                        f[r + DR[k], c + DC[k]] != NOD and f[r + DR[k], c + DC[k]] < f[r, c]
                        for k in range(8))
            assert lower, (r, c)


def test_filled_dem_drains_to_edges():
    """After the fill, D8 leaves NoFlow only on border / coast cells and the
    flow graph is acyclic (the oracle's Kahn order covers every cell)."""
    z = synth.dem(300, 260, seed=2, lambda0=64, ocean=True)
    assert (z == synth.NODATA).mean() >= 0.10
    d = oracle.d8(z)
    rows, cols = z.shape
    nod = d == 9
    coast = np.zeros_like(nod)
    for k in range(8):
        sh = np.zeros_like(nod)
        rs = slice(max(0, -DR[k]), rows - max(0, DR[k]))
        cs = slice(max(0, -DC[k]), cols - max(0, DC[k]))
        rt = slice(max(0, DR[k]), rows - max(0, -DR[k]))
        ct = slice(max(0, DC[k]), cols - max(0, -DC[k]))
        sh[rs, cs] = nod[rt, ct]
        coast |= sh
    border = np.zeros_like(nod)
    border[0, :] = border[-1, :] = border[:, 0] = border[:, -1] = True
    noflow = d == 8
    assert not (noflow & ~(coast | border)).any()
    oracle.accum_u64(d)  # raises on a cycle


def test_generator_is_deterministic():
    a = synth.dem(64, 80, seed=3, lambda0=32, ocean=True)
    b = synth.dem(64, 80, seed=3, lambda0=32, ocean=True)
    np.testing.assert_array_equal(a, b)
    c = synth.dem(64, 80, seed=4, lambda0=32, ocean=True)
    assert not np.array_equal(a, c)


def test_value_noise_amplitude_and_tilt():
    z = synth.value_noise(64, 512, seed=1, lambda0=128, tilt=0.0)
    assert np.abs(z).max() < 100.0
    zt = synth.value_noise(64, 512, seed=1, lambda0=128, tilt=0.01)
    np.testing.assert_allclose(zt - z, np.broadcast_to(0.01 * np.arange(512), z.shape), atol=1e-4)


def test_batch_shapes_distribution():
    shapes = synth.batch_shapes(2000)
    sides = np.array([np.sqrt(r * c) for r, c, *_ in shapes])
    assert 60 <= sides.min() and sides.max() <= 4300
    cells = sum(r * c for r, c, *_ in shapes)
    assert 3.0e9 < cells < 5.5e9
