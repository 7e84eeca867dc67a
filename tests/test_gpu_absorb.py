"""Flow accumulation with absorption (flow_accum_absorb) and its adjoint
(flow_accum_absorb_adjoint) against the oracle's Eq. (1) with alpha per cell
and its transpose: float32 within the float32 parity bound of the float64
oracle, over tile shapes across edges and corners, alpha = 1 (equal to
flow_accum f32 / flow_accum_adjoint) and alpha = 0 (A = w, lambda = g)."""
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_acyclic_dirs(rows, cols, seed, nodata_frac=0.1, noflow_frac=0.02):
    rng = np.random.default_rng(seed)
    z = rng.permutation(rows * cols).astype(np.float32).reshape(rows, cols)
    z[rng.random((rows, cols)) < nodata_frac] = -9999.0
    d = oracle.d8(z)
    d[(rng.random((rows, cols)) < noflow_frac) & (d != 9)] = 8
    return d


def assert_rel(got, want, valid):
    got = got.astype(np.float64)
    pos = valid & (want > 0)
    rel = np.abs(got[pos] - want[pos]) / want[pos]
    assert rel.size == 0 or rel.max() <= F32_RTOL, f"max rel err {rel.max():.3e}"
    assert (got[~valid] == 0).all()


@pytest.mark.parametrize("shape,tile", [((300, 257), (32, 32)), ((130, 200), (64, 48)),
                                        ((97, 64), (16, 64)), ((200, 131), (64, 64)),
                                        ((150, 171), (32, 44)), ((129, 97), (64, 40))])
def test_absorb_matches_oracle(d8m, shape, tile):
    cases = [random_acyclic_dirs(*shape, seed=sum(shape)),
             oracle.d8(synth.dem(*shape, seed=13, lambda0=32, ocean=True))]
    for i, d in enumerate(cases):
        alpha = (0.5 + 0.5 * synth.uniform(d.shape, 70 + i)).astype(np.float32)  # [0.5, 1)
        w = synth.uniform(d.shape, 80 + i)
        want = oracle.accum_absorb_f64(d, alpha, w)
        got = d8m.flow_accum_absorb(dev(d), dev(alpha), dev(w), tile=tile).cpu().numpy()
        assert_rel(got, want, d != 9)
        got1 = d8m.flow_accum_absorb(dev(d), dev(alpha), None, tile=tile).cpu().numpy()
        assert_rel(got1, oracle.accum_absorb_f64(d, alpha), d != 9)


def test_absorb_special_alphas(d8m):
    z = synth.workload_dem("dem512")
    d = oracle.d8(z)
    w = synth.uniform(d.shape, 3)
    one = np.ones(d.shape, np.float32)
    got = d8m.flow_accum_absorb(dev(d), dev(one), dev(w), tile=(64, 48)).cpu().numpy()
    ref = d8m.flow_accum(dev(d), dev(w), acc_type="f32", tile=(64, 48)).cpu().numpy()
    assert_rel(got, ref.astype(np.float64), d != 9)
    zero = np.zeros(d.shape, np.float32)
    got = d8m.flow_accum_absorb(dev(d), dev(zero), dev(w), tile=(64, 48)).cpu().numpy()
    np.testing.assert_array_equal(got, np.where(d != 9, w, 0).astype(np.float32))
    alpha = synth.uniform(d.shape, 4)                                        # [0, 1)
    got = d8m.flow_accum_absorb(dev(d), dev(alpha), dev(w), tile=(64, 48)).cpu().numpy()
    assert_rel(got, oracle.accum_absorb_f64(d, alpha, w), d != 9)


def test_absorb_empty_and_single_tile(d8m):
    e = torch.empty((0, 5), dtype=torch.uint8, device="cuda")
    assert d8m.flow_accum_absorb(e, torch.empty((0, 5), device="cuda")).shape == (0, 5)
    d = random_acyclic_dirs(5, 7, seed=2, nodata_frac=0.0)
    alpha = synth.uniform(d.shape, 5)
    got = d8m.flow_accum_absorb(dev(d), dev(alpha)).cpu().numpy()
    assert_rel(got, oracle.accum_absorb_f64(d, alpha), d != 9)


@pytest.mark.parametrize("shape,tile", [((300, 257), (32, 32)), ((130, 200), (64, 48)),
                                        ((97, 64), (16, 64)), ((200, 131), (64, 64)),
                                        ((150, 171), (32, 44)), ((129, 97), (64, 40))])
def test_absorb_adjoint_matches_oracle(d8m, shape, tile):
    cases = [random_acyclic_dirs(*shape, seed=sum(shape) + 1),
             oracle.d8(synth.dem(*shape, seed=17, lambda0=32, ocean=True))]
    for i, d in enumerate(cases):
        alpha = (0.5 + 0.5 * synth.uniform(d.shape, 90 + i)).astype(np.float32)
        g = synth.uniform(d.shape, 100 + i)
        want = oracle.transpose_absorb_f64(d, alpha, g)
        got = d8m.flow_accum_absorb_adjoint(dev(d), dev(alpha), dev(g), tile=tile).cpu().numpy()
        assert_rel(got, want, d != 9)


def test_absorb_adjoint_special_alphas_and_duality(d8m):
    z = synth.workload_dem("dem512")
    d = oracle.d8(z)
    g = synth.uniform(d.shape, 5)
    one = np.ones(d.shape, np.float32)
    got = d8m.flow_accum_absorb_adjoint(dev(d), dev(one), dev(g), tile=(64, 48)).cpu().numpy()
    ref = d8m.flow_accum_adjoint(dev(d), dev(g), tile=(64, 48)).cpu().numpy()
    assert_rel(got, ref.astype(np.float64), d != 9)
    zero = np.zeros(d.shape, np.float32)
    got = d8m.flow_accum_absorb_adjoint(dev(d), dev(zero), dev(g), tile=(64, 48)).cpu().numpy()
    np.testing.assert_array_equal(got, np.where(d != 9, g, 0).astype(np.float32))
    # <A_alpha(w), g> = <w, lambda_alpha(g)>: the two entry points are transposes
    alpha = synth.uniform(d.shape, 6)
    w = synth.uniform(d.shape, 7)
    A = d8m.flow_accum_absorb(dev(d), dev(alpha), dev(w), tile=(32, 64)).double().cpu().numpy()
    lam = d8m.flow_accum_absorb_adjoint(dev(d), dev(alpha), dev(g), tile=(32, 64)).double().cpu().numpy()
    lhs, rhs = float((A * g).sum()), float((w * lam).sum())
    assert abs(lhs - rhs) <= 1e-4 * abs(lhs)
    assert_rel(lam, oracle.transpose_absorb_f64(d, alpha, g), d != 9)


def test_absorb_adjoint_empty_and_single_tile(d8m):
    e = torch.empty((0, 5), dtype=torch.uint8, device="cuda")
    ef = torch.empty((0, 5), device="cuda")
    assert d8m.flow_accum_absorb_adjoint(e, ef, ef).shape == (0, 5)
    d = random_acyclic_dirs(5, 7, seed=3, nodata_frac=0.0)
    alpha, g = synth.uniform(d.shape, 8), synth.uniform(d.shape, 9)
    got = d8m.flow_accum_absorb_adjoint(dev(d), dev(alpha), dev(g)).cpu().numpy()
    assert_rel(got, oracle.transpose_absorb_f64(d, alpha, g), d != 9)


def test_absorb_autograd(d8m):
    d = oracle.d8(synth.dem(150, 170, seed=21, lambda0=32, ocean=True))
    alpha = synth.uniform(d.shape, 11)
    w = torch.from_numpy(synth.uniform(d.shape, 12)).cuda().requires_grad_(True)
    c = synth.uniform(d.shape, 13)
    A = d8m.FlowAccumAbsorb.apply(w, dev(d), dev(alpha), (32, 48))
    loss = (A * dev(c)).sum()
    loss.backward()
    assert_rel(A.detach().cpu().numpy(), oracle.accum_absorb_f64(d, alpha, w.detach().cpu().numpy()), d != 9)
    assert_rel(w.grad.cpu().numpy(), oracle.transpose_absorb_f64(d, alpha, c), d != 9)


def test_alpha_grad_kernel_exact(d8m):
    # the kernel's only arithmetic is one float32 product A(n) * lambda(receiver(n)):
    # fed the oracle's A and lambda rounded to float32, it must match bit for bit
    for shape, seed in (((97, 131), 31), ((1, 300), 32), ((300, 1), 33)):
        d = random_acyclic_dirs(*shape, seed=seed)
        d[0, 0] = 200                                   # an invalid code: no receiver
        alpha = synth.uniform(d.shape, seed + 1)
        A32 = oracle.accum_absorb_f64(np.where(d == 200, 9, d).astype(np.uint8), alpha).astype(np.float32)
        lam32 = synth.uniform(d.shape, seed + 2)
        r = oracle.receivers(np.where(d == 200, 9, d).astype(np.uint8))
        want = np.zeros(d.shape, np.float32)
        has = r >= 0
        want[has] = A32[has] * lam32.reshape(-1)[r[has]]
        got = d8m.flow_accum_absorb_alpha_grad(dev(d), dev(A32), dev(lam32)).cpu().numpy()
        np.testing.assert_array_equal(got, want)


def test_absorb_autograd_alpha(d8m):
    # A and lambda are each within 1e-4 relative of the oracle, so their
    # product is within (1 + 1e-4)^2 - 1 < 2.1e-4 of the oracle's gradient
    d = oracle.d8(synth.dem(140, 190, seed=23, lambda0=32, ocean=True))
    alpha_np = (0.5 + 0.5 * synth.uniform(d.shape, 14)).astype(np.float32)
    w_np, c = synth.uniform(d.shape, 15), synth.uniform(d.shape, 16)
    w = torch.from_numpy(w_np).cuda().requires_grad_(True)
    alpha = torch.from_numpy(alpha_np).cuda().requires_grad_(True)
    A = d8m.FlowAccumAbsorb.apply(w, dev(d), alpha, (32, 48))
    (A * dev(c)).sum().backward()
    want = oracle.absorb_alpha_grad_f64(d, alpha_np, w_np, c)
    got = alpha.grad.double().cpu().numpy()
    nz = want != 0
    assert (got[~nz] == 0).all()
    rel = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    assert rel.max() <= 2.1e-4, rel.max()
    assert_rel(w.grad.cpu().numpy(), oracle.transpose_absorb_f64(d, alpha_np, c), d != 9)
