"""The D8 kernel's fast choice between the best cardinal drop bc and the best
diagonal drop bd, restated on the host: the diagonal wins when
bd > fma(bc * fl32(sqrt 2), 1 + 2^-20, 2^-126), the cardinal when
bc * fl32(sqrt 2) > fma(bd, 1 + 2^-20, 2^-126) (rho8: bc * t with
t = fl32(2 - r)), otherwise the exact compare decides.  Checked here: every
fast verdict equals the exact one (2 bc^2 against bd^2, or bc t against bd,
in rationals), on random drops over the whole float range (subnormal, tiny,
ordinary, near overflow) and on near-ties, and the fast rule leaves only a
small share of random cells to the exact compare.  The fused multiply-add is
emulated as a float64 computation rounded to float32 (within one float32 ulp
of a single rounding), which the 2^-20 margin absorbs.  (Without the margin
the fast verdict would still be right almost everywhere -- the product is
within about one float32 spacing of the exact value, so no drop lies strictly
between them -- but not provably so across binade edges and underflow; the
margin makes the argument hold everywhere.  A wrong constant or swapped
verdicts fail these tests.)"""
from fractions import Fraction

import numpy as np

K_UP = np.float32(1.0 + 2.0 ** -20)
K_MIN = np.float32(2.0 ** -126)
SQRT2_F = np.float32(np.sqrt(2.0))


def fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def fast_pick(bc, bd, t=None):
    """+1 diagonal, -1 cardinal, 0 left to the exact compare."""
    with np.errstate(over="ignore", invalid="ignore"):
        y = (bc * (SQRT2_F if t is None else t)).astype(np.float32)
        dwin = bd > fma32(y, np.full_like(y, K_UP), np.full_like(y, K_MIN))
        cwin = y > fma32(bd, np.full_like(bd, K_UP), np.full_like(bd, K_MIN))
    assert not np.any(dwin & cwin)
    return np.where(cwin, -1, np.where(dwin, 1, 0))


def exact_pick(bc, bd, t=None):
    out = np.zeros(bc.shape, dtype=np.int64)
    for i, (c, d) in enumerate(zip(bc.tolist(), bd.tolist())):
        fc, fd = Fraction(c), Fraction(d)
        if t is None:
            kc, kd = 2 * fc * fc, fd * fd
        else:
            kc, kd = fc * Fraction(float(t[i])), fd
        out[i] = 1 if kd > kc else (-1 if kc > kd else 0)
    return out


def drops(rng, n):
    """Positive float32 drops spread over every magnitude regime."""
    e = rng.integers(-149, 128, n)
    m = rng.random(n) + 0.5
    with np.errstate(over="ignore"):
        v = np.ldexp(m, e).astype(np.float32)
    v[~np.isfinite(v)] = np.float32(3.0e38)
    v[v == 0] = np.float32(2.0 ** -149)
    return v


def check(bc, bd, t=None):
    f = fast_pick(bc, bd, t)
    decided = f != 0
    e = exact_pick(bc[decided], bd[decided], None if t is None else t[decided])
    assert np.array_equal(f[decided], e), "a fast verdict differs from the exact one"
    return decided.mean()


def test_fast_pick_agrees_with_exact_d8():
    rng = np.random.default_rng(2027)
    n = 20000
    bc, bd = drops(rng, n), drops(rng, n)
    check(bc, bd)
    # near-ties: bd within a few ulps of bc * sqrt 2, in every regime
    base = drops(rng, n)
    near = (base.astype(np.float64) * np.sqrt(2.0) * (1 + rng.integers(-40, 41, n) * 2.0 ** -24))
    with np.errstate(over="ignore"):
        near = near.astype(np.float32)
    ok = np.isfinite(near) & (near > 0)
    check(base[ok], near[ok])
    # ordinary terrain drops (millimetres to metres): nearly every cell decided fast
    bc = (rng.random(n) * 10).astype(np.float32) + np.float32(1e-3)
    bd = (rng.random(n) * 14).astype(np.float32) + np.float32(1e-3)
    assert check(bc, bd) > 0.999


def test_fast_pick_agrees_with_exact_rho8():
    rng = np.random.default_rng(2028)
    n = 20000
    t = (np.float32(2.0) - rng.random(n).astype(np.float32)).astype(np.float32)
    bc, bd = drops(rng, n), drops(rng, n)
    check(bc, bd, t)
    # exact ties bd = bc * t are possible for rho8: the fast rule must leave them
    bc = (rng.integers(1, 1 << 12, n)).astype(np.float32)
    t2 = np.float32(1.5) + np.zeros(n, dtype=np.float32)
    bd = (bc * t2).astype(np.float32)
    assert np.all(fast_pick(bc, bd, t2) == 0)
    assert np.all(exact_pick(bc[:200], bd[:200], t2[:200]) == 0)
