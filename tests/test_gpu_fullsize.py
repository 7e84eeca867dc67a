"""The 32768 x 32768 workload in the launch configuration the benchmark
times (the autotuner's tile shapes for the forward and the adjoint call of
this size class), over the whole raster: D8 codes byte for byte against the
oracle; unit-count accumulation and the float32 adjoint first through
properties that determine them (local balance against the donors, the
adjoint recurrence along receivers, computed here with plain tensor ops,
independently of the library), then every cell against the oracle's Kahn
sweep and its transpose.  Absorption at full size: the same properties and
sampled cells against the oracle's per-cell definitions."""
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
    """Absorption at full size in the benchmark's configuration (32 x 48 tiles,
    alpha ~ U[0.5, 1), U[0, 1) weights and cotangents): local balance
    A(c) = w(c) + sum of alpha(n) A(n) over c's donors and the recurrence
    lambda(c) = g(c) + alpha(c) lambda(receiver) at every cell (float32
    tolerance, as for the plain path), the alpha gradient A(n) lambda(receiver)
    bit for bit, sampled cells against the oracle's per-cell definitions, and
    every cell against the oracle's Kahn-order absorbing forward and its
    transpose (computed on a host thread meanwhile) within 1e-4 relative."""
    dirs = c3["dirs"]
    rows, cols = dirs.shape
    tile = (32, 48)
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
