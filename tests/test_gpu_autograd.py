"""FlowAccum (torch.autograd.Function) with a gauge loss: the gradient with
respect to the weights comes from the HIP adjoint and is checked against the
oracle's transpose solve and against finite differences of the loss computed
by the oracle in float64 (exact for a quadratic loss)."""
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


def gauge_problem(name, n_gauges=64):
    """Workload recipe: gauges are 64 distinct data cells with unit-count
    accumulation >= 1000 (fewer if the raster has fewer such cells), drawn with
    the gauge seed; targets are 1.1 x the accumulation of weights perturbed by
    a factor 0.9 + 0.2 u (perturbation seed)."""
    wl = synth.WORKLOADS[name]
    z = synth.workload_dem(name)
    d = oracle.d8(z)
    w = synth.uniform(d.shape, wl["seed_w"])
    A1 = oracle.accum_u64(d)
    cand = np.flatnonzero((d.ravel() != 9) & (A1.ravel() >= 1000))
    rng = np.random.default_rng(wl["seed_gauges"])
    gauges = np.sort(rng.choice(cand, min(n_gauges, cand.size), replace=False))
    u = synth.uniform(d.shape, wl["seed_perturb"]).astype(np.float64)
    w_pert = w.astype(np.float64) * (0.9 + 0.2 * u)
    t = 1.1 * oracle.accum_f64d(d, w_pert).ravel()[gauges]
    return d, w, gauges, t


def gpu_loss_grad(d8m, d, w, gauges, t, tile=(0, 0)):
    dirs = torch.from_numpy(d).cuda()
    wt = torch.from_numpy(w).cuda().requires_grad_(True)
    A = d8m.FlowAccum.apply(wt, dirs, tile)
    gi = torch.from_numpy(gauges).cuda()
    tt = torch.from_numpy(t.astype(np.float32)).cuda()
    loss = ((A.reshape(-1)[gi] - tt) ** 2).sum()
    loss.backward()
    return A.detach().cpu().numpy(), float(loss.detach()), wt.grad.cpu().numpy()


def test_gauge_loss_gradient_8192(d8m):
    d, w, gauges, t = gauge_problem("gauge8192_ocean")
    assert gauges.size == 64
    A, loss, grad = gpu_loss_grad(d8m, d, w, gauges, t)
    A_ref = oracle.accum_f64(d, w)
    # the forward at every cell, not only through the loss
    valid = d != 9
    pos = valid & (A_ref > 0)
    rel = np.abs(A[pos].astype(np.float64) - A_ref[pos]) / A_ref[pos]
    assert rel.max() <= 1e-4, f"forward max rel err {rel.max():.3e}"
    assert (A[valid & (A_ref == 0)] == 0).all() and (A[~valid] == 0).all()
    res = A_ref.ravel()[gauges] - t
    loss_ref = float((res ** 2).sum())
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    g = np.zeros(d.size, dtype=np.float64)
    g[gauges] = 2.0 * res
    # the oracle transposes the float32-rounded cotangent, as the GPU does
    lam = oracle.transpose_f64(d, g.astype(np.float32).reshape(d.shape))
    valid = d != 9
    scale = np.abs(lam[valid]).max()
    err = np.abs(grad.astype(np.float64) - lam)[valid].max()
    assert err <= 1e-4 * scale, f"normwise {err / scale:.2e}"
    big = valid & (np.abs(lam) >= 1e-3 * scale)
    rel = np.abs(grad[big] - lam[big]) / np.abs(lam[big])
    assert rel.max() <= 1e-4, f"per-cell {rel.max():.2e}"
    assert (grad[~valid] == 0).all()


def test_finite_differences_1024(d8m):
    d, w, gauges, t = gauge_problem("gauge1024_fd")
    _, _, grad = gpu_loss_grad(d8m, d, w, gauges, t, tile=(64, 64))
    w64 = w.astype(np.float64)

    def loss(wv):
        Av = oracle.accum_f64d(d, wv).ravel()
        return float(((Av[gauges] - t) ** 2).sum())

    # cells inside gauge catchments (non-zero gradient) and outside (zero)
    rng = np.random.default_rng(46)
    nz = np.flatnonzero((grad.ravel() != 0))
    zero = np.flatnonzero((grad.ravel() == 0) & (d.ravel() != 9))
    picks = np.concatenate([rng.choice(nz, 24, replace=False), rng.choice(zero, 8, replace=False)])
    scale = np.abs(grad).max()
    for i in picks:
        wp, wm = w64.copy(), w64.copy()
        wp.ravel()[i] += 1.0
        wm.ravel()[i] -= 1.0
        fd = (loss(wp) - loss(wm)) / 2.0  # exact for a quadratic loss (float64)
        assert abs(grad.ravel()[i] - fd) <= 1e-4 * scale, (i, grad.ravel()[i], fd)


def test_flowaccum_forward_matches_flow_accum(d8m):
    z = synth.dem(300, 400, seed=8, lambda0=64, ocean=True)
    d = torch.from_numpy(oracle.d8(z)).cuda()
    w = torch.from_numpy(synth.uniform(z.shape, 9)).cuda()
    a = d8m.FlowAccum.apply(w, d)
    b = d8m.flow_accum(d, w, acc_type="f32")
    assert torch.equal(a, b)


def test_flowaccum_separate_adjoint_tile(d8m):
    # the backward may run on another tile shape than the forward: the same
    # gradient as flow_accum_adjoint on that shape, bit for bit
    z = synth.dem(300, 400, seed=10, lambda0=64, ocean=True)
    d = torch.from_numpy(oracle.d8(z)).cuda()
    w = torch.from_numpy(synth.uniform(z.shape, 11)).cuda().requires_grad_(True)
    c = torch.from_numpy(synth.uniform(z.shape, 12)).cuda()
    a = d8m.FlowAccum.apply(w, d, (64, 44), (64, 32))
    (a * c).sum().backward()
    assert torch.equal(a.detach(), d8m.flow_accum(d, w.detach(), acc_type="f32", tile=(64, 44)))
    assert torch.equal(w.grad, d8m.flow_accum_adjoint(d, c, tile=(64, 32)))
