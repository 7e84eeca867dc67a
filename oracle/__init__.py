"""CPU oracle for D8 flow accumulation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU-baseline
leg may import this package.  The GPU library never links, loads or calls it,
and it shares no code with the GPU library.

Functions (each follows one passage of the paper; see ``oracle.c``):
  d8            D8 steepest descent, exact slope compare, lowest index on ties
  accum_u64     Eq. (1) by the Kahn order of Algorithm 1, 64-bit counts
  accum_f64     Eq. (1) with float32 weights, summed in double
  transpose_f64 the adjoint lambda = (I-P)^-T g (reverse topological sweep)
  rho8          rho8 directions from a per-cell draw r (diagonal distance 2 - r)
  accum_absorb_f64 / transpose_absorb_f64  Eq. (1) with absorption alpha per
                cell, and its transpose
  absorb_alpha_grad_f64  derivative of <c, A> with respect to alpha
  upstream_sum_absorb / downstream_sum_absorb  one value of A / lambda with
                absorption from its definition
  brute_*       path walking, independent of the Kahn order (small inputs)
  upstream_sum  one value of A from its definition (catchment search)
  downstream_sum one value of the adjoint from its definition (path walk)
  tiled         Algorithms 1-3 literally (small inputs), with intermediates
  path_stats    critical-path statistics for a tile shape (sizing only)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

NOFLOW = 8
NODATA = 9
LINK_EXTERNAL = -1
LINK_TERMINATES = -2
LINK_INTERIOR = -3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_ERR = {0: "ok", -1: "bad argument", -4: "invalid direction code", -5: "cycle",
        -6: "overflow", -7: "out of memory"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {_ERR.get(code, '?')}")
        self.code = code


def build() -> str:
    """Compile liboracle.so: plain serial C, no fast-math, no FMA contraction."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math", "-ffp-contract=off",
           "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    lib.orc_d8.argtypes = [vp, vp, i64, i64, ctypes.c_float]
    lib.orc_rho8.argtypes = [vp, vp, vp, i64, i64, ctypes.c_float]
    lib.orc_accum_absorb_f64.argtypes = [vp, i64, i64, vp, i64, vp, vp, vp]
    lib.orc_transpose_absorb_f64.argtypes = [vp, i64, i64, vp, i64, vp, vp, vp]
    lib.orc_receivers.argtypes = [vp, i64, i64, vp]
    lib.orc_accum_u64.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.orc_accum_f64.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.orc_accum_f64d.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.orc_transpose_f64.argtypes = [vp, i64, i64, vp, i64, vp, vp]
    lib.orc_brute_f64.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.orc_brute_u64.argtypes = [vp, i64, i64, vp]
    lib.orc_upstream_sum.argtypes = [vp, i64, i64, vp, i64, i64]
    lib.orc_upstream_sum.restype = ctypes.c_double
    lib.orc_downstream_sum.argtypes = [vp, i64, i64, vp, i64, i64]
    lib.orc_downstream_sum.restype = ctypes.c_double
    lib.orc_upstream_sum_absorb.argtypes = [vp, i64, i64, vp, vp, i64, i64]
    lib.orc_upstream_sum_absorb.restype = ctypes.c_double
    lib.orc_downstream_sum_absorb.argtypes = [vp, i64, i64, vp, vp, i64, i64]
    lib.orc_downstream_sum_absorb.restype = ctypes.c_double
    lib.orc_tiled.argtypes = [vp, i64, i64, i64, i64, vp, vp, vp, vp, vp]
    lib.orc_path_stats.argtypes = [vp, i64, i64, i64, i64, vp]
    for name in ("orc_d8", "orc_receivers", "orc_accum_u64", "orc_accum_f64", "orc_accum_f64d",
                 "orc_transpose_f64", "orc_brute_f64", "orc_brute_u64", "orc_tiled",
                 "orc_path_stats"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check(rc: int):
    if rc != 0:
        raise OracleError(rc)


def _dirs(dirs):
    dirs = np.ascontiguousarray(dirs, dtype=np.uint8)
    assert dirs.ndim == 2
    return dirs


def d8(z: np.ndarray, nodata: float = -9999.0) -> np.ndarray:
    z = np.ascontiguousarray(z, dtype=np.float32)
    out = np.empty(z.shape, dtype=np.uint8)
    _check(_load().orc_d8(_p(z), _p(out), z.shape[0], z.shape[1], ctypes.c_float(nodata)))
    return out


def rho8(z: np.ndarray, rnd: np.ndarray, nodata: float = -9999.0) -> np.ndarray:
    """rho8 directions (orc_rho8): rnd float32 in [0, 1), one draw per cell."""
    z = np.ascontiguousarray(z, dtype=np.float32)
    rnd = np.ascontiguousarray(rnd, dtype=np.float32)
    if rnd.shape != z.shape:
        raise ValueError("rnd and z differ in shape")
    out = np.empty(z.shape, dtype=np.uint8)
    _check(_load().orc_rho8(_p(z), _p(rnd), _p(out), z.shape[0], z.shape[1], ctypes.c_float(nodata)))
    return out


def receivers(dirs: np.ndarray) -> np.ndarray:
    dirs = _dirs(dirs)
    out = np.empty(dirs.shape, dtype=np.int64)
    _check(_load().orc_receivers(_p(dirs), dirs.shape[0], dirs.shape[1], _p(out)))
    return out


def accum_u64(dirs: np.ndarray, w: np.ndarray | None = None, want_order: bool = False):
    dirs = _dirs(dirs)
    A = np.empty(dirs.shape, dtype=np.uint64)
    order = np.empty(dirs.size, dtype=np.int64) if want_order else None
    n = ctypes.c_int64(0)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.uint64)
    _check(_load().orc_accum_u64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(w), _p(A),
                                 _p(order), ctypes.byref(n)))
    return (A, order[: n.value]) if want_order else A


def accum_f64(dirs: np.ndarray, w: np.ndarray | None = None, want_order: bool = False):
    dirs = _dirs(dirs)
    A = np.empty(dirs.shape, dtype=np.float64)
    order = np.empty(dirs.size, dtype=np.int64) if want_order else None
    n = ctypes.c_int64(0)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    _check(_load().orc_accum_f64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(w), _p(A),
                                 _p(order), ctypes.byref(n)))
    return (A, order[: n.value]) if want_order else A


def accum_absorb_f64(dirs: np.ndarray, alpha: np.ndarray, w: np.ndarray | None = None,
                     order: np.ndarray | None = None) -> np.ndarray:
    """Eq. (1) with absorption: A(p) = w(p) + sum over donors n of alpha(n) A(n).
    `order` is accum_u64's Kahn order of the same directions, if at hand."""
    dirs = _dirs(dirs)
    if order is None:
        _, order = accum_u64(dirs, want_order=True)
    alpha = np.ascontiguousarray(alpha, dtype=np.float32)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    A = np.empty(dirs.shape, dtype=np.float64)
    order = np.ascontiguousarray(order, dtype=np.int64)
    _check(_load().orc_accum_absorb_f64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(order), order.size,
                                        _p(w), _p(alpha), _p(A)))
    return A


def transpose_absorb_f64(dirs: np.ndarray, alpha: np.ndarray, g: np.ndarray,
                         order: np.ndarray | None = None) -> np.ndarray:
    """lambda(c) = g(c) + alpha(c) lambda(receiver(c)) (the transpose of accum_absorb_f64).
    `order` is accum_u64's Kahn order of the same directions, if at hand."""
    dirs = _dirs(dirs)
    if order is None:
        _, order = accum_u64(dirs, want_order=True)
    alpha = np.ascontiguousarray(alpha, dtype=np.float32)
    g = np.ascontiguousarray(g, dtype=np.float32)
    lam = np.empty(dirs.shape, dtype=np.float64)
    order = np.ascontiguousarray(order, dtype=np.int64)
    _check(_load().orc_transpose_absorb_f64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(order),
                                            order.size, _p(g), _p(alpha), _p(lam)))
    return lam


def absorb_alpha_grad_f64(dirs: np.ndarray, alpha: np.ndarray, w: np.ndarray | None,
                          c: np.ndarray) -> np.ndarray:
    """d<c, A>/d alpha(n) for A of Eq. (1) with absorption: alpha(n) scales the
    one edge n -> receiver(n), so the derivative is A(n) lambda(receiver(n)),
    lambda = transpose_absorb_f64(c); 0 for cells without a data receiver."""
    A = accum_absorb_f64(dirs, alpha, w)
    lam = transpose_absorb_f64(dirs, alpha, c)
    r = receivers(dirs)
    out = np.zeros(A.shape, dtype=np.float64)
    has = r >= 0
    out[has] = A[has] * lam.reshape(-1)[r[has]]
    return out


def accum_f64d(dirs: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Eq. (1) with float64 weights (used where a weight perturbation must be exact)."""
    dirs = _dirs(dirs)
    A = np.empty(dirs.shape, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    n = ctypes.c_int64(0)
    _check(_load().orc_accum_f64d(_p(dirs), dirs.shape[0], dirs.shape[1], _p(w), _p(A), None,
                                  ctypes.byref(n)))
    return A


def transpose_f64(dirs: np.ndarray, g: np.ndarray, order: np.ndarray | None = None):
    dirs = _dirs(dirs)
    if order is None:
        _, order = accum_u64(dirs, want_order=True)
    g = np.ascontiguousarray(g, dtype=np.float32)
    order = np.ascontiguousarray(order, dtype=np.int64)
    lam = np.empty(dirs.shape, dtype=np.float64)
    _check(_load().orc_transpose_f64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(order),
                                     order.size, _p(g), _p(lam)))
    return lam


def brute_f64(dirs: np.ndarray, w: np.ndarray | None = None, g: np.ndarray | None = None):
    dirs = _dirs(dirs)
    A = np.empty(dirs.shape, dtype=np.float64)
    lam = np.empty(dirs.shape, dtype=np.float64)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    if g is not None:
        g = np.ascontiguousarray(g, dtype=np.float32)
    _check(_load().orc_brute_f64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(w), _p(g), _p(A),
                                 _p(lam)))
    return A, lam


def brute_u64(dirs: np.ndarray) -> np.ndarray:
    dirs = _dirs(dirs)
    A = np.empty(dirs.shape, dtype=np.uint64)
    _check(_load().orc_brute_u64(_p(dirs), dirs.shape[0], dirs.shape[1], _p(A)))
    return A


def upstream_sum(dirs: np.ndarray, r: int, c: int, w: np.ndarray | None = None,
                 max_cells: int = 1 << 40) -> float:
    dirs = _dirs(dirs)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    v = _load().orc_upstream_sum(_p(dirs), dirs.shape[0], dirs.shape[1], _p(w),
                                 r * dirs.shape[1] + c, max_cells)
    if v < 0:
        raise OracleError(-5)
    return v


def downstream_sum(dirs: np.ndarray, r: int, c: int, g: np.ndarray,
                   max_steps: int = 1 << 40) -> float:
    """lambda at (r, c): the sum of g along the cell's downstream path."""
    dirs = _dirs(dirs)
    g = np.ascontiguousarray(g, dtype=np.float32)
    v = _load().orc_downstream_sum(_p(dirs), dirs.shape[0], dirs.shape[1], _p(g),
                                   r * dirs.shape[1] + c, max_steps)
    if v < 0:
        raise OracleError(-5)
    return v


def upstream_sum_absorb(dirs: np.ndarray, r: int, c: int, alpha: np.ndarray,
                        w: np.ndarray | None = None, max_cells: int = 1 << 40) -> float:
    """A at (r, c) with absorption, from its definition: the catchment's w,
    each scaled by the product of alpha along its path to (r, c)."""
    dirs = _dirs(dirs)
    alpha = np.ascontiguousarray(alpha, dtype=np.float32)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    v = _load().orc_upstream_sum_absorb(_p(dirs), dirs.shape[0], dirs.shape[1], _p(w), _p(alpha),
                                        r * dirs.shape[1] + c, max_cells)
    if v < 0:
        raise OracleError(-5)
    return v


def downstream_sum_absorb(dirs: np.ndarray, r: int, c: int, g: np.ndarray, alpha: np.ndarray,
                          max_steps: int = 1 << 40) -> float:
    """lambda at (r, c) with absorption: g along the downstream path, each term
    scaled by the product of alpha over the cells before it."""
    dirs = _dirs(dirs)
    g = np.ascontiguousarray(g, dtype=np.float32)
    alpha = np.ascontiguousarray(alpha, dtype=np.float32)
    v = _load().orc_downstream_sum_absorb(_p(dirs), dirs.shape[0], dirs.shape[1], _p(g), _p(alpha),
                                          r * dirs.shape[1] + c, max_steps)
    if v < 0:
        raise OracleError(-5)
    return v


def tiled(dirs: np.ndarray, th: int, tw: int, w: np.ndarray | None = None):
    """Returns dict(A, Aloc, link, ext) from the literal tiled Algorithms 1-3."""
    dirs = _dirs(dirs)
    A = np.empty(dirs.shape, dtype=np.float64)
    Aloc = np.empty(dirs.shape, dtype=np.float64)
    link = np.empty(dirs.shape, dtype=np.int64)
    ext = np.empty(dirs.shape, dtype=np.float64)
    if w is not None:
        w = np.ascontiguousarray(w, dtype=np.float32)
    _check(_load().orc_tiled(_p(dirs), dirs.shape[0], dirs.shape[1], th, tw, _p(w), _p(A),
                             _p(Aloc), _p(link), _p(ext)))
    return dict(A=A, Aloc=Aloc, link=link, ext=ext)


def path_stats(dirs: np.ndarray, th: int, tw: int) -> dict:
    dirs = _dirs(dirs)
    out = np.zeros(6, dtype=np.int64)
    _check(_load().orc_path_stats(_p(dirs), dirs.shape[0], dirs.shape[1], th, tw, _p(out)))
    keys = ("max_in_tile_run", "max_crossings", "perimeter_cells", "exit_cells",
            "entry_cells", "longest_path")
    return dict(zip(keys, (int(v) for v in out)))
