"""The 32768 x 32768 workload in the launch configuration the benchmark
times (the autotuner's tile shapes for the forward and the adjoint call of
this size class), over the whole raster: D8 codes byte for byte against the
oracle; unit-count accumulation and the float32 adjoint first through
properties that determine them (local balance against the donors, the
adjoint recurrence along receivers, computed here with plain tensor ops,
independently of the library), then every cell against the oracle's Kahn
sweep and its transpose.  Absorption at full size: the same properties,
sampled cells against the oracle's per-cell definitions and every cell
against the oracle.  rho8 codes over the whole raster, and a raster past 2^31
cells."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DR = (-1, -1, -1, 0, 0, 1, 1, 1)
DC = (-1, 0, 1, -1, 1, -1, 0, 1)


@pytest.fixture(scope="module")
def d8m():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    import paper_1608_04431_amd as m
    m._lib.load()
    return m


def receivers(dirs: torch.Tensor) -> torch.Tensor:
    """Flat receiver index per cell, -1 where there is none (NoFlow, NoData,
    off the raster, or into NoData)."""
    rows, cols = dirs.shape
    k = dirs.long()
    r = torch.arange(rows, device=dirs.device).view(-1, 1).expand(rows, cols)
    c = torch.arange(cols, device=dirs.device).view(1, -1).expand(rows, cols)
    dr = torch.tensor(DR + (0, 0), device=dirs.device)[k.clamp(max=9)]
    dc = torch.tensor(DC + (0, 0), device=dirs.device)[k.clamp(max=9)]
    nr, nc = r + dr, c + dc
    ok = (k < 8) & (nr >= 0) & (nr < rows) & (nc >= 0) & (nc < cols)
    idx = (nr.clamp(0, rows - 1) * cols + nc.clamp(0, cols - 1))
    ok &= dirs.view(-1)[idx.view(-1)].view(rows, cols) != 9
    return torch.where(ok, idx, torch.full_like(idx, -1)).view(-1)


@pytest.fixture(scope="module")
def dem32768():
    z = synth.workload_dem("dem32768")
    return z


@pytest.fixture(scope="module")
def c3(d8m, dem32768):
    """The GPU's D8 codes of the 32768^2 workload and the oracle's, and the
    oracle's unit counts (with their Kahn order) and transpose with the
    benchmark's cotangent, then its absorbing forward and transpose (alpha
    ~ U[0.5, 1), the cotangent raster as weights and as cotangent) on the
    same order, computed on a host thread while the GPU tests run (the
    oracle is serial C; the thread only overlaps its calls)."""
    wl = synth.WORKLOADS["dem32768"]
    z = dem32768
    pool = ThreadPoolExecutor(max_workers=1)
    d_ref_f = pool.submit(oracle.d8, z)
    dirs = d8m.d8_directions(torch.from_numpy(z).cuda())
    g_host = synth.uniform(z.shape, wl["seed_g"])
    alpha_host = (0.5 + 0.5 * synth.uniform(z.shape, wl["seed_g"] + 1)).astype(np.float32)
    d_ref = d_ref_f.result()
    kahn = {}

    def solve():
        A, kahn["order"] = oracle.accum_u64(d_ref, want_order=True)
        lam = oracle.transpose_f64(d_ref, g_host, kahn["order"])
        return A, lam

    def solve_absorb():
        order = kahn.pop("order")
        A = oracle.accum_absorb_f64(d_ref, alpha_host, g_host, order=order)
        lam = oracle.transpose_absorb_f64(d_ref, alpha_host, g_host, order=order)
        return A, lam

    ref_f = pool.submit(solve)
    ref_absorb_f = pool.submit(solve_absorb)
    yield dict(dirs=dirs, d_ref=d_ref, g_host=g_host, alpha_host=alpha_host, ref=ref_f,
               ref_absorb=ref_absorb_f)
    pool.shutdown(wait=True)


@pytest.mark.timeout(900)
def test_dem32768_d8_whole_raster(c3):
    """D8 codes byte for byte over the whole raster."""
    np.testing.assert_array_equal(c3["dirs"].cpu().numpy(), c3["d_ref"])


@pytest.mark.timeout(900)
def test_dem32768_full_size(d8m, c3):
    """Unit counts and the float32 adjoint on the benchmark's tile shapes:
    first through properties that determine them (local balance, the
    adjoint recurrence), then every cell against the oracle: counts bit for
    bit, the adjoint within 1e-4 relative (dense cotangent U[0, 1), so
    lambda >= g > 0 wherever g > 0)."""
    wl = synth.WORKLOADS["dem32768"]
    dirs = c3["dirs"]
    rows, cols = dirs.shape
    from paper_1608_04431_amd.autotune import Tuner
    tuner = Tuner()
    tile_f, tile_a = tuner.tile_for(rows, cols, kind="fwd"), tuner.tile_for(rows, cols, kind="adj")
    A = d8m.flow_accum(dirs, acc_type="u32", tile=tile_f)
    g = torch.from_numpy(c3["g_host"]).cuda()
    lam = d8m.flow_accum_adjoint(dirs, g, tile=tile_a)
    torch.cuda.synchronize()
    # the same forward and adjoint with the raster in host memory, streamed
    # in bands: counts bit for bit, the adjoint (tiles recomputed, exits
    # seeded) within float32 rounding of the in-memory one
    dirs_h = dirs.cpu().pin_memory()
    As = d8m.flow_accum_streamed(dirs_h, tile=tile_f)
    assert torch.equal(As, A.cpu())
    del As
    g_h = g.cpu().pin_memory()
    Ls = d8m.flow_accum_adjoint_streamed(dirs_h, g_h, tile=tile_a).double()
    Lm = lam.cpu().double()
    assert float(((Ls - Lm).abs() / Lm.abs().clamp_min(1e-30)).max()) <= 1e-5
    del Ls, Lm
    # the float32 weighted forward (weights = the cotangent raster): the
    # streamed call equals the in-memory one bit for bit (fixed-order sums)
    Af = d8m.flow_accum(dirs, g, acc_type="f32", tile=tile_f)
    Afs = d8m.flow_accum_streamed_f32(dirs_h, g_h, tile=tile_f)
    assert torch.equal(Afs, Af.cpu())
    del Af, Afs, g_h, dirs_h

    recv = receivers(dirs)
    data = dirs.view(-1) != 9
    has = recv >= 0
    # local balance, exact in int64: A(c) = 1 + sum of A over c's donors
    A64 = A.view(-1).long() & 0xFFFFFFFF
    inflow = torch.zeros_like(A64)
    inflow.index_add_(0, recv[has], A64[has])
    assert torch.equal(A64[data], 1 + inflow[data])
    assert (A64[~data] == 0).all()
    # the outlets hold every data cell once
    assert int(A64[data & ~has].sum()) == int(data.sum())
    del inflow, A64

    # adjoint recurrence lambda(c) = g(c) + lambda(receiver), float32 tolerance
    L = lam.view(-1).double()
    G = g.view(-1).double()
    down = torch.zeros_like(L)
    down[has] = L[recv[has]]
    res = (L - G - down)[data].abs()
    scale = (L.abs() + down.abs())[data]
    assert (res <= 1e-4 * scale + 1e-6).all(), float((res / (scale + 1e-30)).max())
    assert (L[~data] == 0).all()
    del L, G, down, res, scale, recv, has, data

    # every cell against the oracle
    A_host = A.cpu().numpy().view(np.uint32)
    L_host = lam.cpu().numpy()
    del A, lam, g
    A_ref, lam_ref = c3["ref"].result()
    assert A_ref.max() < 2 ** 32
    bad = np.flatnonzero(A_host.ravel() != A_ref.ravel())
    assert bad.size == 0, f"{bad.size} cells differ, first at {divmod(int(bad[0]), cols)}"
    del A_ref, A_host
    valid = c3["d_ref"].ravel() != 9
    pos = valid & (lam_ref.ravel() > 0)
    want = lam_ref.ravel()[pos]
    rel = np.abs(L_host.ravel()[pos].astype(np.float64) - want) / want
    assert rel.max() <= 1e-4, f"adjoint max rel err {rel.max():.3e}"
    zero = valid & (lam_ref.ravel() == 0)
    assert (L_host.ravel()[zero] == 0).all() and (L_host.ravel()[~valid] == 0).all()


@pytest.mark.timeout(900)
def test_dem32768_absorb_full_size(d8m, c3):
    """Absorption at full size in the benchmark's configuration (48 x 32 tiles,
    alpha ~ U[0.5, 1), U[0, 1) weights and cotangents): local balance
    A(c) = w(c) + sum of alpha(n) A(n) over c's donors and the recurrence
    lambda(c) = g(c) + alpha(c) lambda(receiver) at every cell (float32
    tolerance, as for the plain path), the alpha gradient A(n) lambda(receiver)
    bit for bit, sampled cells against the oracle's per-cell definitions, and
    every cell against the oracle's Kahn-order absorbing forward and its
    transpose (computed on a host thread meanwhile) within 1e-4 relative."""
    dirs = c3["dirs"]
    rows, cols = dirs.shape
    tile = (48, 32)
    w_host, alpha_host, d_host = c3["g_host"], c3["alpha_host"], c3["d_ref"]
    w, alpha = torch.from_numpy(w_host).cuda(), torch.from_numpy(alpha_host).cuda()
    A = d8m.flow_accum_absorb(dirs, alpha, w, tile=tile)
    lam = d8m.flow_accum_absorb_adjoint(dirs, alpha, w, tile=tile)
    ga = d8m.flow_accum_absorb_alpha_grad(dirs, A, lam)
    torch.cuda.synchronize()

    recv = receivers(dirs)
    data = dirs.view(-1) != 9
    has = recv >= 0
    Ad, Wd, Al = A.view(-1).double(), w.view(-1).double(), alpha.view(-1).double()
    inflow = torch.zeros_like(Ad)
    inflow.index_add_(0, recv[has], Al[has] * Ad[has])
    res = (Ad - Wd - inflow)[data].abs()
    scale = (Ad.abs() + inflow.abs())[data]
    assert (res <= 1e-4 * scale + 1e-6).all(), float((res / (scale + 1e-30)).max())
    assert (Ad[~data] == 0).all()
    del inflow, res, scale

    L = lam.view(-1).double()
    down = torch.zeros_like(L)
    down[has] = Al[has] * L[recv[has]]
    res = (L - Wd - down)[data].abs()
    scale = (L.abs() + down.abs())[data]
    assert (res <= 1e-4 * scale + 1e-6).all(), float((res / (scale + 1e-30)).max())
    assert (L[~data] == 0).all()
    del down, res, scale, Ad, Wd, L

    # dL/dalpha(n) = A(n) lambda(receiver(n)): one float32 product
    want = torch.zeros_like(A.view(-1))
    want[has] = A.view(-1)[has] * lam.view(-1)[recv[has]]
    assert torch.equal(ga.view(-1), want)
    del want, ga

    gen = torch.Generator(device="cuda").manual_seed(12)
    cand = torch.randint(0, rows * cols, (4096,), device="cuda", generator=gen)
    picks = cand[data[cand]][:30].tolist()
    A_host, L_host = A.cpu().numpy(), lam.cpu().numpy()
    for i in picks:
        r, c = divmod(int(i), cols)
        want = oracle.upstream_sum_absorb(d_host, r, c, alpha_host, w_host)
        assert abs(A_host[r, c] - want) <= 1e-4 * max(want, 1e-6), (r, c, A_host[r, c], want)
        want = oracle.downstream_sum_absorb(d_host, r, c, w_host, alpha_host)
        assert abs(L_host[r, c] - want) <= 1e-4 * max(want, 1e-6), (r, c, L_host[r, c], want)
    del A, lam, w, alpha, dirs, recv, data, has

    # every cell against the oracle (weights and cotangents in [0, 1), so
    # both results are >= 0 and zero exactly where the oracle's are)
    A_ref, lam_ref = c3["ref_absorb"].result()
    valid = d_host.ravel() != 9
    for got, want_all, name in ((A_host, A_ref, "forward"), (L_host, lam_ref, "adjoint")):
        got, want_all = got.ravel(), want_all.ravel()
        pos = valid & (want_all > 0)
        rel = np.abs(got[pos].astype(np.float64) - want_all[pos]) / want_all[pos]
        assert rel.max() <= 1e-4, f"{name} max rel err {rel.max():.3e}"
        zero = valid & (want_all == 0)
        assert (got[zero] == 0).all() and (got[~valid] == 0).all(), name
        del rel, pos, zero


def receivers_band(dirs: torch.Tensor, r0: int, r1: int) -> torch.Tensor:
    """receivers() for rows r0 .. r1 - 1 of `dirs` (flat indices into the
    whole raster), so that the checks below stay within memory at any size."""
    rows, cols = dirs.shape
    k = dirs[r0:r1].long()
    r = torch.arange(r0, r1, device=dirs.device).view(-1, 1).expand(r1 - r0, cols)
    c = torch.arange(cols, device=dirs.device).view(1, -1).expand(r1 - r0, cols)
    dr = torch.tensor(DR + (0, 0), device=dirs.device)[k.clamp(max=9)]
    dc = torch.tensor(DC + (0, 0), device=dirs.device)[k.clamp(max=9)]
    nr, nc = r + dr, c + dc
    ok = (k < 8) & (nr >= 0) & (nr < rows) & (nc >= 0) & (nc < cols)
    idx = nr.clamp(0, rows - 1) * cols + nc.clamp(0, cols - 1)
    ok &= dirs.view(-1)[idx.view(-1)].view(r1 - r0, cols) != 9
    return torch.where(ok, idx, torch.full_like(idx, -1)).view(-1)


@pytest.mark.timeout(900)
def test_over_2p31_cells(d8m):
    """A raster of 44001 x 53688 = 2.36e9 cells, past 2^31 (flat indices
    cross it at row 40000), ragged against the tile shapes in both
    directions, in the launch configuration of its size class: D8 codes on
    windows (the last rows among them) against the oracle, then unit counts
    and the float32 adjoint through local balance, outlet mass and the
    adjoint recurrence at every cell, the streamed forward and adjoint equal
    to the in-memory calls, the same properties for absorption
    (alpha ~ U[0.5, 1), the cotangent raster as weights and cotangent), and
    sampled cells past index 2^31 against the oracle's per-cell definitions.  The DEM (a tilted surface
    with long waves, seeded noise and NoData discs) is made on the device:
    the terrain generator would take minutes at this size."""
    rows, cols = 44001, 53688
    n = rows * cols
    assert n > 2 ** 31 + 2 ** 27
    gen = torch.Generator(device="cuda").manual_seed(2031)
    z = torch.empty(rows, cols, dtype=torch.float32, device="cuda")
    band = 4096
    for r0 in range(0, rows, band):
        r1 = min(rows, r0 + band)
        rr = torch.arange(r0, r1, device="cuda", dtype=torch.float32).view(-1, 1)
        cc = torch.arange(cols, device="cuda", dtype=torch.float32).view(1, -1)
        zb = 0.002 * rr + 0.001 * cc + 3.0 * torch.sin(rr / 300.0) * torch.sin(cc / 450.0)
        zb += 0.01 * torch.rand(r1 - r0, cols, device="cuda", generator=gen)
        z[r0:r1] = zb
        del zb
    for (rc, ccen, rad) in ((1000, 2000, 300), (20000, 30000, 900), (41000, 50000, 700), (43990, 100, 60)):
        a0, a1, b0, b1 = max(0, rc - rad), min(rows, rc + rad), max(0, ccen - rad), min(cols, ccen + rad)
        rr = torch.arange(a0, a1, device="cuda").view(-1, 1)
        cc = torch.arange(b0, b1, device="cuda").view(1, -1)
        disc = (rr - rc) ** 2 + (cc - ccen) ** 2 < rad * rad
        z[a0:a1, b0:b1][disc] = -9999.0
    dirs = d8m.d8_directions(z)
    torch.cuda.synchronize()

    # D8 on windows: each window plus a one-cell margin (clipped to the
    # raster) through the oracle; the window's cells have all their
    # neighbours inside the margin or off the raster
    for (w0, w1, v0, v1) in ((0, 300, 0, 700), (20500, 20800, 29000, 30300), (40900, 41200, 49000, 50700),
                             (43700, rows, cols - 900, cols), (39990, 40010, 0, cols)):
        e0, e1, f0, f1 = max(0, w0 - 1), min(rows, w1 + 1), max(0, v0 - 1), min(cols, v1 + 1)
        want = oracle.d8(z[e0:e1, f0:f1].cpu().numpy())[w0 - e0:w1 - e0, v0 - f0:v1 - f0]
        np.testing.assert_array_equal(dirs[w0:w1, v0:v1].cpu().numpy(), want, err_msg=f"window {w0}:{w1}")

    from paper_1608_04431_amd.autotune import Tuner
    tuner = Tuner()
    tile_f, tile_a = tuner.tile_for(rows, cols, kind="fwd"), tuner.tile_for(rows, cols, kind="adj")
    assert rows % tile_f[0] and cols % tile_f[1] and rows % tile_a[0] and cols % tile_a[1]
    A = d8m.flow_accum(dirs, acc_type="u32", tile=tile_f)
    g = torch.rand(rows, cols, device="cuda", generator=gen)
    lam = d8m.flow_accum_adjoint(dirs, g, tile=tile_a)
    torch.cuda.synchronize()

    Av, Lv, Gv, Dv = A.view(-1), lam.view(-1), g.view(-1), dirs.view(-1)
    inflow = torch.zeros(n, dtype=torch.int64, device="cuda")
    outlet_mass, data_cells = 0, 0
    step = 2048
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        s = slice(r0 * cols, r1 * cols)
        recv = receivers_band(dirs, r0, r1)
        has = recv >= 0
        data = Dv[s] != 9
        A64 = Av[s].long() & 0xFFFFFFFF
        inflow.index_add_(0, recv[has], A64[has])
        outlet_mass += int(A64[data & ~has].sum())
        data_cells += int(data.sum())
        # adjoint recurrence lambda(c) = g(c) + lambda(receiver), float32 tolerance
        L = Lv[s].double()
        down = torch.zeros_like(L)
        down[has] = Lv[recv[has]].double()
        res = (L - Gv[s].double() - down)[data].abs()
        scale = (L.abs() + down.abs())[data]
        assert (res <= 1e-4 * scale + 1e-6).all(), (r0, float((res / (scale + 1e-30)).max()))
        assert (L[~data] == 0).all()
        del recv, has, data, A64, L, down, res, scale
    # the outlets hold every data cell once
    assert outlet_mass == data_cells
    for r0 in range(0, rows, step):
        s = slice(r0 * cols, min(rows, r0 + step) * cols)
        data = Dv[s] != 9
        A64 = Av[s].long() & 0xFFFFFFFF
        assert torch.equal(A64[data], 1 + inflow[s][data]), r0
        assert (A64[~data] == 0).all()
    del inflow

    # the same calls with the raster in host memory, streamed in bands: counts
    # bit for bit, the adjoint within float32 rounding of the in-memory one
    dirs_h = dirs.cpu().pin_memory()
    As = d8m.flow_accum_streamed(dirs_h, tile=tile_f)
    assert torch.equal(As, A.cpu())
    del As
    g_h = g.cpu().pin_memory()
    Ls = d8m.flow_accum_adjoint_streamed(dirs_h, g_h, tile=tile_a)
    Lm = lam.cpu()
    assert float(((Ls.double() - Lm.double()).abs() / Lm.double().abs().clamp_min(1e-30)).max()) <= 1e-5
    del Ls, Lm, g_h, dirs_h

    # absorption at the same size (its own per-node and per-cell arrays):
    # local balance and the adjoint recurrence at every cell
    alpha = 0.5 + 0.5 * torch.rand(rows, cols, device="cuda", generator=gen)
    Ab = d8m.flow_accum_absorb(dirs, alpha, g)
    Lb = d8m.flow_accum_absorb_adjoint(dirs, alpha, g)
    torch.cuda.synchronize()
    Abv, Lbv, Alv = Ab.view(-1), Lb.view(-1), alpha.view(-1)
    inflow = torch.zeros(n, dtype=torch.float64, device="cuda")
    for r0 in range(0, rows, step):
        s = slice(r0 * cols, min(rows, r0 + step) * cols)
        recv = receivers_band(dirs, r0, min(rows, r0 + step))
        has = recv >= 0
        data = Dv[s] != 9
        inflow.index_add_(0, recv[has], (Alv[s][has].double() * Abv[s][has].double()))
        L = Lbv[s].double()
        down = torch.zeros_like(L)
        down[has] = Alv[s][has].double() * Lbv[recv[has]].double()
        res = (L - Gv[s].double() - down)[data].abs()
        scale = (L.abs() + down.abs())[data]
        assert (res <= 1e-4 * scale + 1e-6).all(), ("absorb adjoint", r0)
        assert (L[~data] == 0).all()
        del recv, has, data, L, down, res, scale
    for r0 in range(0, rows, step):
        s = slice(r0 * cols, min(rows, r0 + step) * cols)
        data = Dv[s] != 9
        Ad = Abv[s].double()
        res = (Ad - Gv[s].double() - inflow[s])[data].abs()
        scale = (Ad.abs() + inflow[s].abs())[data]
        assert (res <= 1e-4 * scale + 1e-6).all(), ("absorb forward", r0)
        assert (Ad[~data] == 0).all()
    del inflow, Ab, Lb, alpha, Abv, Lbv, Alv

    # sampled cells past 2^31 (and a few before) against the per-cell
    # definitions: catchment search for A, downstream path sum for lambda
    d_host = dirs.cpu().numpy()
    g_host = g.cpu().numpy()
    cand = torch.randint(2 ** 31, n, (4096,), device="cuda", generator=gen)
    cand = torch.cat([cand, torch.randint(0, 2 ** 31, (1024,), device="cuda", generator=gen)])
    ok = (Dv[cand] != 9) & ((Av[cand].long() & 0xFFFFFFFF) < 200000)
    picks = cand[ok][:24].tolist() + cand[ok][-8:].tolist()
    assert sum(i >= 2 ** 31 for i in picks) >= 20
    for i in picks:
        r, c = divmod(int(i), cols)
        assert int(A[r, c].item()) & 0xFFFFFFFF == int(oracle.upstream_sum(d_host, r, c)), (r, c)
        want = oracle.downstream_sum(d_host, r, c, g_host)
        got = float(lam[r, c].item())
        assert abs(got - want) <= 1e-4 * max(want, 1e-6), (r, c, got, want)


@pytest.mark.timeout(900)
def test_dem32768_rho8_whole_raster(d8m, dem32768):
    """rho8 directions (one U[0, 1) draw per cell) over the whole 32768^2
    raster, code for code against the oracle (run on a host thread
    meanwhile); then unit counts over them through local balance and outlet
    mass at every cell (rho8, like D8, sends each cell to a strictly lower
    neighbour, so its directions are acyclic)."""
    rows, cols = dem32768.shape
    rnd = synth.uniform((rows, cols), 77)
    pool = ThreadPoolExecutor(max_workers=1)
    ref = pool.submit(oracle.rho8, dem32768, rnd)
    dirs = d8m.d8_directions_rho8(torch.from_numpy(dem32768).cuda(), torch.from_numpy(rnd).cuda())
    from paper_1608_04431_amd.autotune import Tuner
    A = d8m.flow_accum(dirs, acc_type="u32", tile=Tuner().tile_for(rows, cols, kind="fwd"))
    torch.cuda.synchronize()
    got = dirs.cpu().numpy()
    want = ref.result()
    pool.shutdown(wait=True)
    bad = np.flatnonzero(got.ravel() != want.ravel())
    assert bad.size == 0, f"{bad.size} codes differ, first at {divmod(int(bad[0]), cols)}"
    del got, want, rnd

    Dv, Av = dirs.view(-1), A.view(-1)
    inflow = torch.zeros(rows * cols, dtype=torch.int64, device="cuda")
    outlet_mass, data_cells = 0, 0
    step = 4096
    for r0 in range(0, rows, step):
        s = slice(r0 * cols, min(rows, r0 + step) * cols)
        recv = receivers_band(dirs, r0, min(rows, r0 + step))
        has = recv >= 0
        data = Dv[s] != 9
        A64 = Av[s].long() & 0xFFFFFFFF
        inflow.index_add_(0, recv[has], A64[has])
        outlet_mass += int(A64[data & ~has].sum())
        data_cells += int(data.sum())
    assert outlet_mass == data_cells
    for r0 in range(0, rows, step):
        s = slice(r0 * cols, min(rows, r0 + step) * cols)
        data = Dv[s] != 9
        A64 = Av[s].long() & 0xFFFFFFFF
        assert torch.equal(A64[data], 1 + inflow[s][data]), r0
        assert (A64[~data] == 0).all()
