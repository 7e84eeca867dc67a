"""Batches of rasters (flow_accum_batched, d8_graph_*): every raster's
results equal the single-raster calls with the same tile shape bit for bit
(the same tile code runs, and the cross-tile sums are exact or done in the
same order), and agree with the oracle; a recorded graph replays correctly
with other work between replays and with inputs changed in place."""
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


# uneven shapes (thin, tiny, ragged against the tiles) and per-raster tiles
SHAPES = [((300, 420), (64, 64)), ((64, 64), (64, 64)), ((37, 53), (32, 48)), ((1, 70), (0, 0)),
          ((70, 1), (0, 0)), ((513, 257), (64, 32)), ((129, 200), (50, 37)), ((256, 96), (32, 32)),
          ((0, 40), (0, 0)), ((90, 600), (48, 64)), ((2, 2), (0, 0)), ((200, 200), (16, 64))]


def make_rasters(d8m, seed0=100):
    out = []
    for i, ((rows, cols), tile) in enumerate(SHAPES):
        if rows == 0 or cols == 0:
            z = np.zeros((rows, cols), np.float32)
        else:
            z = synth.dem(rows, cols, seed=seed0 + i, lambda0=max(16, max(rows, cols) // 8))
        d = oracle.d8(z) if z.size else np.zeros((rows, cols), np.uint8)
        w = synth.uniform((rows, cols), 6000 + i)
        g = synth.uniform((rows, cols), 7000 + i)
        out.append((d, w, g, tile))
    return out


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def single(d8m, d, w, g, tile):
    dd, wd, gd = to_dev(d), to_dev(w), to_dev(g)
    if d.size == 0:
        return np.zeros(d.shape, np.float32), np.zeros(d.shape, np.float32)
    a = d8m.flow_accum(dd, wd, acc_type="f32", tile=tile)
    lam = d8m.flow_accum_adjoint(dd, gd, tile=tile)
    return a.cpu().numpy(), lam.cpu().numpy()


def test_batch_equals_single_calls_and_oracle(d8m):
    data = make_rasters(d8m)
    rasters = [d8m.Raster(to_dev(d), to_dev(w), to_dev(g), tile=t) for d, w, g, t in data]
    b = d8m.Batch(rasters, "fwd+adj")
    b.run()
    b.check_status()
    for (d, w, g, t), r in zip(data, rasters):
        a1, l1 = single(d8m, d, w, g, t)
        np.testing.assert_array_equal(r.acc.cpu().numpy(), a1, err_msg=f"acc {d.shape} {t}")
        np.testing.assert_array_equal(r.grad_weights.cpu().numpy(), l1, err_msg=f"lam {d.shape} {t}")
    # every raster against the oracle, per cell: float32 forward within 1e-4
    # relative of the float64 sums (exactly 0 where they are 0), the adjoint of
    # the dense cotangent U[0, 1) likewise
    for (d, w, g, t), r in zip(data, rasters):
        if d.size == 0:
            continue
        valid = d != 9
        for got, want, what in ((r.acc, oracle.accum_f64(d, w), "acc"),
                                (r.grad_weights, oracle.transpose_f64(d, g), "lam")):
            got = got.cpu().numpy().astype(np.float64)
            pos = valid & (want > 0)
            rel = np.abs(got[pos] - want[pos]) / want[pos]
            assert rel.size == 0 or rel.max() <= 1e-4, f"{what} {d.shape} {t}: {rel.max():.3e}"
            assert (got[valid & (want == 0)] == 0).all() and (got[~valid] == 0).all()


def test_batch_modes_separately(d8m):
    data = make_rasters(d8m, seed0=300)[:6]
    fw = [d8m.Raster(to_dev(d), to_dev(w), tile=t) for d, w, g, t in data]
    d8m.Batch(fw, "fwd").run()
    ad = [d8m.Raster(to_dev(d), None, to_dev(g), tile=t) for d, w, g, t in data]
    d8m.Batch(ad, "adj").run()
    for (d, w, g, t), rf, ra in zip(data, fw, ad):
        a1, l1 = single(d8m, d, w, g, t)
        np.testing.assert_array_equal(rf.acc.cpu().numpy(), a1)
        np.testing.assert_array_equal(ra.grad_weights.cpu().numpy(), l1)


def test_batch_unit_weights_match_counts(d8m):
    d = oracle.d8(synth.dem(333, 190, seed=9, lambda0=64))
    r = d8m.Raster(to_dev(d), None, tile=(64, 64))
    d8m.Batch([r], "fwd").run()
    want = oracle.accum_u64(d).astype(np.float64)
    np.testing.assert_array_equal(r.acc.cpu().numpy().astype(np.float64), want)


def test_graph_replays(d8m):
    data = make_rasters(d8m, seed0=500)
    rasters = [d8m.Raster(to_dev(d), to_dev(w), to_dev(g), tile=t) for d, w, g, t in data]
    b = d8m.Batch(rasters, "fwd+adj")
    b.run()
    torch.cuda.synchronize()
    eager = [(r.acc.clone(), r.grad_weights.clone()) for r in rasters]
    graph = b.graph()
    try:
        for rep in range(4):
            for r in rasters:
                r.acc.fill_(-1.0)
                r.grad_weights.fill_(-1.0)
            # unrelated eager work on the same stream between replays
            junk = torch.randn(1 << 20, device="cuda").sum()
            graph.launch()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            b.check_status()
            for r, (a, lam) in zip(rasters, eager):
                assert torch.equal(r.acc, a), f"replay {rep}"
                assert torch.equal(r.grad_weights, lam), f"replay {rep}"
        # inputs are read at replay time
        for (d, w, g, t), r in zip(data, rasters):
            r.weights.mul_(0.5)
            r.grad_acc.add_(1.0)
        graph.launch()
        torch.cuda.synchronize()
        for (d, w, g, t), r in zip(data, rasters):
            a1, l1 = single(d8m, d, w * np.float32(0.5), g + np.float32(1.0), t)
            np.testing.assert_array_equal(r.acc.cpu().numpy(), a1)
            np.testing.assert_array_equal(r.grad_weights.cpu().numpy(), l1)
    finally:
        graph.destroy()


def test_batch_reports_data_errors(d8m):
    good = oracle.d8(synth.dem(100, 100, seed=3, lambda0=32))
    bad = good.copy()
    bad[10, 10] = 200                         # invalid code
    rs = [d8m.Raster(to_dev(good), None, tile=(32, 32)), d8m.Raster(to_dev(bad), None, tile=(32, 32))]
    b = d8m.Batch(rs, "fwd")
    b.run()
    with pytest.raises(d8m.D8Error, match="invalid direction"):
        b.check_status()
    cyc = np.full((40, 40), 6, np.uint8)
    cyc[20, 20], cyc[21, 20] = 6, 1           # two cells pointing at each other
    rs = [d8m.Raster(to_dev(cyc), None, torch.zeros(40, 40, device="cuda"), tile=(16, 16))]
    b = d8m.Batch(rs, "fwd+adj")
    b.run()
    with pytest.raises(d8m.D8Error, match="cycle"):
        b.check_status()
