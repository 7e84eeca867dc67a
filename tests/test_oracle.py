"""Pins for the CPU oracle: each check ties an oracle function to something
other than itself -- hand-computed fixtures, brute force, closed forms,
invariants, an independent exact-arithmetic D8 and the exactness of finite
differences on a quadratic loss.  CPU only."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from conftest import GOLDEN_FILES, load_golden

DR = [-1, -1, -1, 0, 0, 1, 1, 1]
DC = [-1, 0, 1, -1, 1, -1, 0, 1]


# ------------------------------------------------------------ helpers --------
def random_acyclic_dirs(rows, cols, seed, nodata_frac=0.1, noflow_frac=0.02):
    """D8 on distinct random elevations is acyclic (every step strictly
    descends).  NoData cells and forced NoFlow cells keep it acyclic."""
    rng = np.random.default_rng(seed)
    z = rng.permutation(rows * cols).astype(np.float32).reshape(rows, cols)
    z[rng.random((rows, cols)) < nodata_frac] = -9999.0
    d = oracle.d8(z)
    d[(rng.random((rows, cols)) < noflow_frac) & (d != 9)] = 8
    return d


def py_receiver(d, r, c):
    """Independent restatement of the receiver rule for the Python checks."""
    k = int(d[r, c])
    if k >= 8:
        return None
    rr, cc = r + DR[k], c + DC[k]
    if not (0 <= rr < d.shape[0] and 0 <= cc < d.shape[1]) or d[rr, cc] == 9:
        return None
    return rr, cc


# ------------------------------------------------------------ P1 fixtures ----
@pytest.mark.parametrize("name", GOLDEN_FILES)
def test_golden_untiled(name):
    dirs, A_hand, _ = load_golden(name)
    A = oracle.accum_u64(dirs)
    np.testing.assert_array_equal(A, A_hand)
    Af = oracle.accum_f64(dirs)
    np.testing.assert_array_equal(Af, A_hand.astype(np.float64))
    np.testing.assert_array_equal(oracle.brute_u64(dirs), A_hand)


@pytest.mark.parametrize("name", GOLDEN_FILES)
def test_golden_tiled(name):
    dirs, A_hand, tile = load_golden(name)
    tiles = [tile] if tile else []
    tiles += [(1, 1), (2, 2), (1, 3), (dirs.shape[0], dirs.shape[1])]
    for th, tw in tiles:
        T = oracle.tiled(dirs, th, tw)
        np.testing.assert_array_equal(T["A"], A_hand.astype(np.float64), err_msg=f"{th}x{tw}")


def test_corner_tiles_intermediates():
    """Hand-derived intermediates of the literal tiled scheme on the corner
    fixture (tiles 2x2): the diagonal crossing at the tile corner is a
    FlowExternal exit whose inflow lands on the diagonal neighbour."""
    dirs, _, (th, tw) = load_golden("corner_tiles.txt")
    T = oracle.tiled(dirs, th, tw)
    # (1,1) leaves its tile directly: FlowExternal with A_loc = 2
    assert T["link"][1, 1] == oracle.LINK_EXTERNAL
    assert T["Aloc"][1, 1] == 2
    # (0,0) links to the exit cell (1,1)
    assert T["link"][0, 0] == 1 * 4 + 1
    # (2,2) receives 2 across the corner; its own A_loc is 1
    assert T["ext"][2, 2] == 2 and T["Aloc"][2, 2] == 1
    # a NoFlow perimeter cell terminates
    assert T["link"][0, 1] == oracle.LINK_TERMINATES


def test_reentry_intermediates():
    dirs, _, (th, tw) = load_golden("reentry_tiles.txt")
    T = oracle.tiled(dirs, th, tw)
    # tile A: (0,0) -> (0,2) which exits east
    assert T["link"][0, 0] == 0 * 6 + 2
    assert T["link"][0, 2] == oracle.LINK_EXTERNAL and T["Aloc"][0, 2] == 3
    # tile B: (0,3) -> (1,3) exits west; its cross inflow is 3
    assert T["ext"][0, 3] == 3 and T["Aloc"][1, 3] == 2
    # back in tile A: (1,2) receives 5 from (1,3)
    assert T["ext"][1, 2] == 5
    # (2,3) receives 9 from (2,2)
    assert T["ext"][2, 3] == 9


# ------------------------------------------------------------ P2 brute -------
@pytest.mark.parametrize("seed", range(6))
def test_kahn_equals_brute_force(seed):
    rows, cols = [(1, 40), (40, 1), (17, 23), (64, 64), (31, 5), (50, 61)][seed]
    d = random_acyclic_dirs(rows, cols, seed)
    np.testing.assert_array_equal(oracle.accum_u64(d), oracle.brute_u64(d))
    w = synth.uniform((rows, cols), 100 + seed)
    g = synth.uniform((rows, cols), 200 + seed)
    A_b, lam_b = oracle.brute_f64(d, w, g)
    A_k = oracle.accum_f64(d, w)
    np.testing.assert_allclose(A_k, A_b, rtol=1e-12, atol=0)
    lam = oracle.transpose_f64(d, g)
    np.testing.assert_allclose(lam, lam_b, rtol=1e-12, atol=0)


def test_kahn_pure_python_tiny():
    """A third, dictionary-based restatement of Eq. (1) on a tiny field."""
    d = random_acyclic_dirs(9, 11, 7)
    rows, cols = d.shape
    memo = {}

    def A(r, c):
        if (r, c) in memo:
            return memo[(r, c)]
        s = 1
        for k in range(8):
            rr, cc = r + DR[k], c + DC[k]
            if 0 <= rr < rows and 0 <= cc < cols and d[rr, cc] != 9 and \
                    py_receiver(d, rr, cc) == (r, c):
                s += A(rr, cc)
        memo[(r, c)] = s
        return s

    want = np.array([[A(r, c) if d[r, c] != 9 else 0 for c in range(cols)] for r in range(rows)],
                    dtype=np.uint64)
    np.testing.assert_array_equal(oracle.accum_u64(d), want)


# ------------------------------------------------------------ P3 invariants --
@pytest.mark.parametrize("seed", range(3))
def test_invariants(seed):
    d = random_acyclic_dirs(80, 90, 30 + seed)
    w = synth.uniform(d.shape, 40 + seed)
    A = oracle.accum_u64(d).astype(np.int64)
    Af = oracle.accum_f64(d, w)
    rec = oracle.receivers(d)
    valid = d != 9
    outlets = valid & (rec.reshape(d.shape) < 0)
    # mass balance: what leaves through the outlets is everything that fell
    assert A[outlets].sum() == valid.sum()
    np.testing.assert_allclose(Af[outlets].sum(), w[valid].astype(np.float64).sum(), rtol=1e-12)
    # local balance: A(c) - w(c) - sum of donors = 0
    inflow = np.zeros(d.size, dtype=np.int64)
    inflow_f = np.zeros(d.size)
    src = np.nonzero(rec.ravel() >= 0)[0]
    np.add.at(inflow, rec.ravel()[src], A.ravel()[src])
    np.add.at(inflow_f, rec.ravel()[src], Af.ravel()[src])
    bal = A.ravel() - valid.ravel() - inflow
    assert (bal[valid.ravel()] == 0).all()
    np.testing.assert_allclose(Af.ravel()[valid.ravel()],
                               (w.ravel().astype(np.float64) + inflow_f)[valid.ravel()],
                               rtol=1e-12)
    assert (A[valid] >= 1).all() and (A[~valid] == 0).all()


def test_cycle_and_bad_code_detected():
    d = np.array([[4, 3]], dtype=np.uint8)  # east <-> west: a 2-cycle
    with pytest.raises(oracle.OracleError) as e:
        oracle.accum_u64(d)
    assert e.value.code == -5
    with pytest.raises(oracle.OracleError) as e:
        oracle.brute_u64(d)
    assert e.value.code == -5
    with pytest.raises(oracle.OracleError) as e:
        oracle.tiled(d, 1, 1)
    assert e.value.code == -5
    with pytest.raises(oracle.OracleError) as e:
        oracle.accum_u64(np.array([[4, 10]], dtype=np.uint8))
    assert e.value.code == -4


# ------------------------------------------------------------ P4 closed forms
def test_tilted_plane_closed_form():
    rows, cols = 37, 53
    z = (0.01 * np.arange(cols, dtype=np.float64))[None, :].repeat(rows, 0).astype(np.float32)
    d = oracle.d8(z)
    assert (d[:, 1:] == 3).all()          # everything flows west
    assert (d[:, 0] == 8).all()           # column 0 has no lower neighbour
    A = oracle.accum_u64(d)
    want = np.broadcast_to(cols - np.arange(cols), (rows, cols))
    np.testing.assert_array_equal(A, want)


def test_valley_closed_form():
    rows, cols, c0 = 29, 41, 17
    r_ = np.arange(rows, dtype=np.float64)[:, None]
    c_ = np.arange(cols, dtype=np.float64)[None, :]
    z = (0.01 * np.abs(c_ - c0) + 0.001 * r_).astype(np.float32)
    d = oracle.d8(z)
    A = oracle.accum_u64(d).astype(np.int64)
    want = np.zeros((rows, cols), dtype=np.int64)
    for r in range(rows):
        for c in range(cols):
            if c < c0:
                want[r, c] = c + 1
            elif c > c0:
                want[r, c] = cols - c
            else:
                want[r, c] = (rows - r) * cols
    np.testing.assert_array_equal(A, want)


# ------------------------------------------------------------ P5 tiled -------
@pytest.mark.parametrize("seed", range(4))
def test_tiled_equals_untiled(seed):
    rows, cols = [(64, 64), (45, 77), (100, 37), (3, 200)][seed]
    d = random_acyclic_dirs(rows, cols, 300 + seed)
    w = synth.uniform(d.shape, 400 + seed)
    A = oracle.accum_u64(d).astype(np.float64)
    Af = oracle.accum_f64(d, w)
    for th, tw in [(1, 1), (1, 5), (5, 1), (7, 9), (16, 16), (13, 64), (rows, cols)]:
        T = oracle.tiled(d, th, tw)
        np.testing.assert_array_equal(T["A"], A, err_msg=f"tile {th}x{tw}")
        Tw = oracle.tiled(d, th, tw, w)
        np.testing.assert_allclose(Tw["A"], Af, rtol=1e-12, err_msg=f"tile {th}x{tw}")


def test_tiled_on_synthetic_terrain():
    z = synth.dem(256, 192, seed=9, lambda0=64, ocean=False)
    d = oracle.d8(z)
    A = oracle.accum_u64(d).astype(np.float64)
    for th, tw in [(32, 32), (64, 16), (100, 100)]:
        np.testing.assert_array_equal(oracle.tiled(d, th, tw)["A"], A)


# ------------------------------------------------------------ P6 adjoint -----
def test_adjoint_dot_product_identity_exact():
    d = random_acyclic_dirs(60, 70, 11)
    rng = np.random.default_rng(12)
    w = rng.integers(0, 50, d.shape).astype(np.float32)
    g = rng.integers(-30, 30, d.shape).astype(np.float32)
    A = oracle.accum_f64(d, w)
    lam = oracle.transpose_f64(d, g)
    valid = d != 9
    lhs = float((g.astype(np.float64) * A)[valid].sum())
    rhs = float((lam * w.astype(np.float64))[valid].sum())
    assert lhs == rhs  # small integers: exact in double


def test_adjoint_unit_cotangent_is_catchment():
    d = random_acyclic_dirs(40, 40, 13, nodata_frac=0.05)
    A = oracle.accum_u64(d)
    rng = np.random.default_rng(14)
    valid = np.argwhere(d != 9)
    for r, c in valid[rng.choice(len(valid), 10, replace=False)]:
        g = np.zeros(d.shape, dtype=np.float32)
        g[r, c] = 1.0
        lam = oracle.transpose_f64(d, g)
        assert set(np.unique(lam)) <= {0.0, 1.0}
        assert lam.sum() == A[r, c]


# ------------------------------------------------------------ P7 FD ----------
def test_finite_difference_exact_on_quadratic_loss():
    """L(w) = sum_k (A_k - t_k)^2 is quadratic in w, so the central difference
    equals dL/dw_i exactly for any step; checked at h = 1 in double."""
    z = synth.dem(96, 80, seed=41, lambda0=32, ocean=False)
    d = oracle.d8(z)
    w = synth.uniform(d.shape, 42).astype(np.float64)
    A = oracle.accum_f64d(d, w)
    rng = np.random.default_rng(44)
    valid = np.flatnonzero(d.ravel() != 9)
    gauges = rng.choice(valid, 8, replace=False)
    t = 1.1 * A.ravel()[gauges]

    def loss(wv):
        Av = oracle.accum_f64d(d, wv).ravel()
        return float(((Av[gauges] - t) ** 2).sum())

    g = np.zeros(d.size, dtype=np.float64)
    g[gauges] = 2.0 * (A.ravel()[gauges] - t)
    lam = oracle.transpose_f64(d, g.astype(np.float32).reshape(d.shape))
    # cotangent entries are not exact in float32; use a relative bound that
    # the float32 rounding of g admits, plus exactness of FD in double
    for i in rng.choice(valid, 12, replace=False):
        wp, wm = w.copy(), w.copy()
        wp.ravel()[i] += 1.0
        wm.ravel()[i] -= 1.0
        fd = (loss(wp) - loss(wm)) / 2.0
        # exact gradient in double: sum of g over the gauges on i's flow path
        path_sum = 0.0
        r, c = divmod(int(i), d.shape[1])
        while True:
            path_sum += g[r * d.shape[1] + c]
            nxt = py_receiver(d, r, c)
            if nxt is None:
                break
            r, c = nxt
        assert abs(fd - path_sum) <= 1e-9 * max(1.0, abs(path_sum))
        assert abs(lam.ravel()[i] - path_sum) <= 1e-6 * max(1.0, abs(path_sum))


# ------------------------------------------------------------ P8 D8 ----------
def exact_d8(z, nodata=-9999.0):
    """D8 written again with exact rationals: slope^2 = d^2 (cardinal) or
    d^2 / 2 (diagonal) where d is the float32 drop; largest wins, lowest index
    on ties, NoFlow if no strictly lower valid neighbour, 9 for NoData."""
    rows, cols = z.shape
    out = np.zeros(z.shape, dtype=np.uint8)
    for r in range(rows):
        for c in range(cols):
            zc = z[r, c]
            if zc == np.float32(nodata) or np.isnan(zc):
                out[r, c] = 9
                continue
            best, best_s = 8, Fraction(0)
            for k in range(8):
                rr, cc = r + DR[k], c + DC[k]
                if not (0 <= rr < rows and 0 <= cc < cols):
                    continue
                zn = z[rr, cc]
                if zn == np.float32(nodata) or np.isnan(zn):
                    continue
                dd = Fraction(float(np.float32(zc) - np.float32(zn)))
                if dd <= 0:
                    continue
                s = dd * dd if (DR[k] == 0 or DC[k] == 0) else dd * dd / 2
                if s > best_s:
                    best, best_s = k, s
            out[r, c] = best
    return out


@pytest.mark.parametrize("seed", range(4))
def test_d8_exact_ties_integer_dem(seed):
    rng = np.random.default_rng(500 + seed)
    z = rng.integers(0, 4, (23, 29)).astype(np.float32)  # many exact ties
    z[rng.random(z.shape) < 0.05] = -9999.0
    z[0, 0] = np.nan
    np.testing.assert_array_equal(oracle.d8(z), exact_d8(z))


def test_d8_random_floats_and_terrain():
    rng = np.random.default_rng(77)
    z = (rng.random((31, 37)) * 10).astype(np.float32)
    np.testing.assert_array_equal(oracle.d8(z), exact_d8(z))
    t = synth.dem(40, 50, seed=5, lambda0=16, ocean=False)
    np.testing.assert_array_equal(oracle.d8(t), exact_d8(t))


def test_d8_near_sqrt2_boundary():
    # diagonal drops within a few ulps of sqrt(2) times the cardinal drop, for
    # drops from subnormal to 1e38: the slope compare must be exact
    z = synth.sqrt2_blocks()
    got = oracle.d8(z)
    np.testing.assert_array_equal(got, exact_d8(z))
    centres = got[1, 1::3]
    assert (centres == 1).any() and (centres == 2).any()


def exact_rho8(z, rnd, nodata=-9999.0):
    """rho8 again with exact rationals: slope = d / 1 (cardinal) or
    d / t (diagonal) with t = fl32(2 - r) of the cell and d the float32 drop;
    largest wins, lowest index on ties."""
    rows, cols = z.shape
    out = np.zeros(z.shape, dtype=np.uint8)
    for r in range(rows):
        for c in range(cols):
            zc = z[r, c]
            if zc == np.float32(nodata) or np.isnan(zc):
                out[r, c] = 9
                continue
            t = Fraction(float(np.float32(2.0) - np.float32(rnd[r, c])))
            best, best_s = 8, Fraction(0)
            for k in range(8):
                rr, cc = r + DR[k], c + DC[k]
                if not (0 <= rr < rows and 0 <= cc < cols):
                    continue
                zn = z[rr, cc]
                if zn == np.float32(nodata) or np.isnan(zn):
                    continue
                d = Fraction(float(np.float32(zc) - np.float32(zn)))
                if d <= 0:
                    continue
                s = d if (DR[k] == 0 or DC[k] == 0) else d / t
                if s > best_s:
                    best, best_s = k, s
            out[r, c] = best
    return out


def test_rho8_exact_on_terrain_and_ties():
    rng = np.random.default_rng(91)
    z = rng.integers(0, 5, (21, 27)).astype(np.float32)     # many tied drops
    z[rng.random(z.shape) < 0.05] = -9999.0
    rnd = synth.uniform(z.shape, 3)
    np.testing.assert_array_equal(oracle.rho8(z, rnd), exact_rho8(z, rnd))
    t = synth.dem(30, 41, seed=8, lambda0=12, ocean=True)
    rnd = synth.uniform(t.shape, 4)
    got = oracle.rho8(t, rnd)
    np.testing.assert_array_equal(got, exact_rho8(t, rnd))
    # r = 0 everywhere: t = 2, diagonal slopes halved; r -> 1: t -> 1
    for rv in (0.0, np.nextafter(np.float32(1), np.float32(0))):
        rr = np.full(t.shape, rv, np.float32)
        np.testing.assert_array_equal(oracle.rho8(t, rr), exact_rho8(t, rr))


def test_rho8_half_blocks_closed_form():
    # diagonal drop 1.5, cardinal 1: the diagonal wins iff 1.5 / (2 - r) > 1,
    # i.e. r > 1/2; r = 1/2 is a tie and the lower index (north) wins
    rv = np.array([0.0, 0.25, 0.4999999, 0.5, 0.5000001, 0.75, 0.9999999], np.float32)
    z, r = synth.rho8_half_blocks(rv)
    got = oracle.rho8(z, r)[1, 1::3]
    want = np.where(rv > 0.5, 2, 1)
    np.testing.assert_array_equal(got, want)
    # over many uniform draws the diagonal share is the share of r above 1/2
    rv = synth.uniform((1, 4000), 12)[0]
    z, r = synth.rho8_half_blocks(rv)
    got = oracle.rho8(z, r)[1, 1::3]
    np.testing.assert_array_equal(got == 2, rv > 0.5)
    assert abs((got == 2).mean() - 0.5) < 0.03


def test_d8_tie_breaks_lowest_index():
    # centre 1, all eight neighbours 0: cardinal slope 1 beats diagonal 1/sqrt2;
    # of the four cardinals (N=1, W=3, E=4, S=6) the lowest index N wins
    z = np.zeros((3, 3), dtype=np.float32)
    z[1, 1] = 1.0
    assert oracle.d8(z)[1, 1] == 1
    # only diagonals lower: NW (0) wins among equals
    z = np.ones((3, 3), dtype=np.float32)
    z[1, 1] = 2.0
    z[0, 0] = z[0, 2] = z[2, 0] = z[2, 2] = 0.0
    z[0, 1] = z[1, 0] = z[1, 2] = z[2, 1] = 2.0
    assert oracle.d8(z)[1, 1] == 0


# ------------------------------------------------------------ spot values ----
def test_downstream_sum_matches_transpose_and_brute_force():
    rng = np.random.default_rng(77)
    for seed in range(3):
        z = rng.permutation(30 * 41).astype(np.float32).reshape(30, 41)
        z[rng.random(z.shape) < 0.1] = -9999.0
        d = oracle.d8(z)
        g = rng.random(d.shape).astype(np.float32)
        lam = oracle.transpose_f64(d, g)
        _, lam_b = oracle.brute_f64(d, g=g)
        for r, c in zip(rng.integers(0, 30, 40), rng.integers(0, 41, 40)):
            v = oracle.downstream_sum(d, int(r), int(c), g)
            assert abs(v - lam[r, c]) <= 1e-12 * max(1.0, lam[r, c])
            assert abs(v - lam_b[r, c]) <= 1e-12 * max(1.0, lam[r, c])
    # hand case: a row flowing east sums g from the cell to the east edge
    d = np.full((1, 5), 4, np.uint8)
    g = np.array([[1, 2, 4, 8, 16]], np.float32)
    assert [oracle.downstream_sum(d, 0, c, g) for c in range(5)] == [31, 30, 28, 24, 16]
    cyc = np.array([[4, 3]], np.uint8)   # two cells pointing at each other
    with pytest.raises(oracle.OracleError):
        oracle.downstream_sum(cyc, 0, 0, np.ones((1, 2), np.float32), max_steps=10)


def test_upstream_sum_matches_kahn():
    d = random_acyclic_dirs(50, 50, 21)
    w = synth.uniform(d.shape, 22)
    A = oracle.accum_u64(d)
    Af = oracle.accum_f64(d, w)
    for r, c in [(0, 0), (10, 20), (49, 49), (25, 3)]:
        assert oracle.upstream_sum(d, r, c) == A[r, c]
        assert abs(oracle.upstream_sum(d, r, c, w) - Af[r, c]) <= 1e-12 * max(1, Af[r, c])


# ------------------------------------------------------------ path stats -----
def test_path_stats_hand():
    # a 1x8 row flowing east in 1x4 tiles: in-tile runs of 4, one crossing,
    # perimeter = every cell (tiles 1 cell high), 1 exit (col 3) and 1 entry (col 4)
    d = np.full((1, 8), 4, dtype=np.uint8)
    s = oracle.path_stats(d, 1, 4)
    assert s == dict(max_in_tile_run=4, max_crossings=1, perimeter_cells=8, exit_cells=1,
                     entry_cells=1, longest_path=8)


# ------------------------------------------------------------ absorption ----
def py_absorb_brute(d, w, alpha):
    """A(x) = sum over cells y whose path passes x of w(y) times the product
    of alpha over the path's cells before x (path walking, no Kahn order)."""
    A = np.zeros(d.shape)
    for r in range(d.shape[0]):
        for c in range(d.shape[1]):
            if d[r, c] == 9:
                continue
            v, cell = float(w[r, c]), (r, c)
            while cell is not None:
                A[cell] += v
                v *= float(alpha[cell])
                cell = py_receiver(d, *cell)
    return A


def test_absorb_reduces_to_eq1_and_to_w():
    d = random_acyclic_dirs(23, 31, 7)
    w = synth.uniform(d.shape, 5)
    valid = d != 9
    one = np.ones(d.shape, np.float32)
    np.testing.assert_array_equal(oracle.accum_absorb_f64(d, one, w), oracle.accum_f64(d, w))
    zero = np.zeros(d.shape, np.float32)
    np.testing.assert_array_equal(oracle.accum_absorb_f64(d, zero, w), np.where(valid, w, 0.0))
    g = synth.uniform(d.shape, 6)
    np.testing.assert_array_equal(oracle.transpose_absorb_f64(d, one, g), oracle.transpose_f64(d, g))
    np.testing.assert_array_equal(oracle.transpose_absorb_f64(d, zero, g), np.where(valid, g, 0.0))


def test_absorb_brute_force_and_duality():
    d = random_acyclic_dirs(17, 19, 8)
    w = synth.uniform(d.shape, 9)
    alpha = synth.uniform(d.shape, 10)
    A = oracle.accum_absorb_f64(d, alpha, w)
    np.testing.assert_allclose(A, py_absorb_brute(d, w, alpha), rtol=1e-12, atol=1e-12)
    # transpose: <g, A(w)> = <lambda(g), w> (one linear operator and its adjoint)
    g = synth.uniform(d.shape, 11)
    lam = oracle.transpose_absorb_f64(d, alpha, g)
    assert abs(float((g.astype(np.float64) * A).sum()) - float((lam * w).sum())) < 1e-9 * A.sum()


def test_absorb_chain_closed_form():
    # a row flowing east: A at position k (0-based) = sum_{j<=k} a^j
    d = np.full((1, 12), 4, np.uint8)
    d[0, -1] = 8
    for a in (0.25, 0.5, 0.9):
        alpha = np.full(d.shape, a, np.float32)
        A = oracle.accum_absorb_f64(d, alpha)
        want = np.array([sum(float(np.float32(a)) ** j for j in range(k + 1)) for k in range(12)])
        np.testing.assert_allclose(A[0], want, rtol=1e-14)


def test_absorb_alpha_grad_central_differences():
    # <c, A_alpha(w)> is affine in each single alpha(n): every flow path passes
    # n at most once, so alpha(n) enters each path product at most once.  A
    # central difference is then exact; alpha +- h are exact in float32.
    d = random_acyclic_dirs(11, 13, 21)
    rng = np.random.default_rng(22)
    alpha = (rng.integers(8, 57, d.shape) / 64.0).astype(np.float32)
    w = synth.uniform(d.shape, 23)
    c = synth.uniform(d.shape, 24)
    grad = oracle.absorb_alpha_grad_f64(d, alpha, w, c)
    h = 0.125
    for n in range(d.size):
        ap, am = alpha.copy(), alpha.copy()
        ap.flat[n] += h
        am.flat[n] -= h
        fd = (float((c * oracle.accum_absorb_f64(d, ap, w)).sum()) -
              float((c * oracle.accum_absorb_f64(d, am, w)).sum())) / (2 * h)
        assert abs(fd - grad.flat[n]) <= 1e-12 * max(1.0, abs(fd)), n
    # no data receiver (NoData, NoFlow, off the raster): no dependence on alpha
    r = oracle.receivers(d)
    assert (grad[r < 0] == 0).all()
    assert (grad[(r >= 0) & (d != 9)] != 0).any()


def test_absorb_alpha_grad_chain_closed_form():
    # a row flowing east into a NoFlow cell, w = 1, c = e_last: A(k) = sum_{j<=k} a^j,
    # lambda(m) = a^(last - m), so dA(last)/d alpha(k) = A(k) a^(last - k - 1)
    n = 9
    d = np.full((1, n), 4, np.uint8)
    d[0, -1] = 8
    a = np.float32(0.75)
    alpha = np.full(d.shape, a, np.float32)
    c = np.zeros(d.shape, np.float32)
    c[0, -1] = 1
    grad = oracle.absorb_alpha_grad_f64(d, alpha, None, c)[0]
    af = float(a)
    for k in range(n - 1):
        Ak = sum(af ** j for j in range(k + 1))
        assert abs(grad[k] - Ak * af ** (n - 2 - k)) < 1e-14
    assert grad[-1] == 0


def test_absorb_per_cell_definitions():
    # catchment search with alpha products / downstream path sum with alpha
    # prefixes, independent of the Kahn order, at every cell
    d = random_acyclic_dirs(19, 23, 31)
    alpha = synth.uniform(d.shape, 32)
    w, g = synth.uniform(d.shape, 33), synth.uniform(d.shape, 34)
    A = oracle.accum_absorb_f64(d, alpha, w)
    lam = oracle.transpose_absorb_f64(d, alpha, g)
    A1 = oracle.accum_absorb_f64(d, alpha)
    for r in range(d.shape[0]):
        for c in range(d.shape[1]):
            assert abs(oracle.upstream_sum_absorb(d, r, c, alpha, w) - A[r, c]) <= 1e-12 * max(1.0, A[r, c])
            assert abs(oracle.upstream_sum_absorb(d, r, c, alpha) - A1[r, c]) <= 1e-12 * max(1.0, A1[r, c])
            assert abs(oracle.downstream_sum_absorb(d, r, c, g, alpha) - lam[r, c]) <= 1e-12 * max(1.0, lam[r, c])
