"""Seeded synthetic inputs for the flow-accumulation workloads.

This module prepares inputs only and holds none of the method's arithmetic
(no flow directions, no accumulation).  It is shared by the CPU oracle's
tests, the GPU parity tests and the benchmark, so both sides see identical
inputs.

Terrain recipe (stands in for the paper's SRTM / NED / PAMAP tiles, which are
not available here):
  * 6-octave value noise, amplitude 100 m, base wavelength ``lambda0`` cells,
    lattice values from a SplitMix64 counter hash of (seed, octave, i, j),
    smoothstep-blended;
  * a planar tilt of 0.01 m per column (regional fall toward column 0);
  * optional NoData "ocean" discs (radius 50..500 cells at 8192^2, scaled down
    for smaller rasters) until >= 10 % of the raster is NoData;
  * elevations quantised to integer millimetres and depression-filled with a
    Priority-Flood + epsilon (epsilon = 1 mm), so every data cell drains to the
    border or a coast.
Weights and cotangents are float32 uniform in [0, 1) from numpy's PCG64
(``numpy.random.default_rng(seed)``).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

NODATA = np.float32(-9999.0)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None


def build() -> str:
    """Compile libsynth.so (host C, OpenMP)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", _LIB_PATH, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    f32p = ctypes.POINTER(ctypes.c_float)
    lib.syn_value_noise.argtypes = [f32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.syn_value_noise.restype = None
    lib.syn_ocean_mask.argtypes = [f32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double]
    lib.syn_ocean_mask.restype = ctypes.c_int64
    lib.syn_fill_dem.argtypes = [f32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32]
    lib.syn_fill_dem.restype = ctypes.c_int
    lib.syn_fill_int.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.c_int64,
                                 ctypes.c_int32]
    lib.syn_fill_int.restype = ctypes.c_int
    _lib = lib
    return lib


def _fp(a: np.ndarray):
    assert a.dtype == np.float32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def value_noise(rows: int, cols: int, seed: int, lambda0: float, octaves: int = 6,
                amp: float = 100.0, tilt: float = 0.01) -> np.ndarray:
    z = np.empty((rows, cols), dtype=np.float32)
    _load().syn_value_noise(_fp(z), rows, cols, seed, float(lambda0), octaves, amp, tilt)
    return z


def ocean_mask(z: np.ndarray, seed: int, frac: float = 0.10, rmin: float = 50.0,
               rmax: float = 500.0) -> int:
    """Mark NoData discs in place until ``frac`` of the cells are NoData."""
    return int(_load().syn_ocean_mask(_fp(z), z.shape[0], z.shape[1], seed, frac, rmin, rmax))


def fill(z: np.ndarray, eps_mm: int = 1) -> np.ndarray:
    """Quantise to mm and Priority-Flood + epsilon fill, in place."""
    rc = _load().syn_fill_dem(_fp(z), z.shape[0], z.shape[1], eps_mm)
    if rc != 0:
        raise MemoryError("syn_fill_dem failed")
    return z


def fill_int(zi: np.ndarray, eps: int) -> np.ndarray:
    """Priority-Flood + epsilon on an int32 raster (INT32_MIN = NoData), in place."""
    assert zi.dtype == np.int32 and zi.flags.c_contiguous
    rc = _load().syn_fill_int(zi.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              zi.shape[0], zi.shape[1], eps)
    if rc != 0:
        raise MemoryError("syn_fill_int failed")
    return zi


def dem(rows: int, cols: int, seed: int, lambda0: float, ocean: bool = False,
        filled: bool = True) -> np.ndarray:
    """A filled float32 DEM (metres); NoData cells hold ``NODATA``."""
    z = value_noise(rows, cols, seed, lambda0)
    if ocean:
        # disc radii 50..500 cells at 8192^2 and above; scaled down for smaller
        # rasters so a single disc cannot swallow most of the raster
        rmax = min(500.0, max(rows, cols) / 16.0)
        ocean_mask(z, seed, rmin=rmax / 10.0, rmax=rmax)
    if filled:
        fill(z)
    return z


def uniform(shape, seed: int) -> np.ndarray:
    """float32 U[0,1) weights / cotangents from PCG64."""
    return np.random.default_rng(seed).random(shape, dtype=np.float32)


# ---------------------------------------------------------------- workloads
# Named by content.  ``lambda0`` is the base noise wavelength in cells.
WORKLOADS = {
    "dem512": dict(rows=512, cols=512, seed=1, lambda0=128, ocean=False),
    "dem8192_ocean": dict(rows=8192, cols=8192, seed=2, lambda0=1024, ocean=True, seed_w=21),
    "dem32768": dict(rows=32768, cols=32768, seed=3, lambda0=4096, ocean=False, seed_g=31),
    "gauge8192_ocean": dict(rows=8192, cols=8192, seed=4, lambda0=1024, ocean=True, seed_w=42,
                            seed_gauges=44, seed_perturb=45),
    "gauge1024_fd": dict(rows=1024, cols=1024, seed=41, lambda0=128, ocean=True, seed_w=42,
                         seed_gauges=44, seed_perturb=45),
}


def workload_dem(name: str) -> np.ndarray:
    w = WORKLOADS[name]
    return dem(w["rows"], w["cols"], w["seed"], w["lambda0"], ocean=w["ocean"])


def batch_shapes(n: int = 2000, seed: int = 55, smin: int = 64, smax: int = 4096):
    """Uneven DEM sizes: side s log-uniform in [smin, smax], aspect a uniform in
    [0.5, 2]; rows = round(s*sqrt(a)), cols = round(s/sqrt(a)).  Returns a list of
    (rows, cols, lambda0, dem_seed, w_seed, g_seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        s = math.exp(rng.uniform(math.log(smin), math.log(smax)))
        a = rng.uniform(0.5, 2.0)
        rows = max(1, int(round(s * math.sqrt(a))))
        cols = max(1, int(round(s / math.sqrt(a))))
        lam = max(16, int(round(max(rows, cols) / 8)))
        out.append((rows, cols, lam, 5000 + i, 6000 + i, 7000 + i))
    return out


def sqrt2_blocks() -> np.ndarray:
    """3 x 3k float32 raster of independent 3 x 3 blocks for the D8 slope
    compare at its hardest: each block's centre is 0, its north neighbour
    -dc and its north-east neighbour -dd, with dd within a few float32 ulps
    of dc * sqrt(2) (and the other neighbours far higher), for drops dc from
    subnormal to 1e38.  Input only: no direction is computed here."""
    pairs = []
    for dc in (1.0, 3.7e-3, 0.125, 7.0, 1e-29, 2e-30, 1e-40, 1e20, 9e36, 2e37, 1e38):
        dc = np.float32(dc)
        mid = np.float32(float(dc) * 2.0 ** 0.5)
        dd = mid
        for _ in range(6):
            dd = np.nextafter(dd, np.float32(0))
        for _ in range(13):
            if np.isfinite(dd):
                pairs.append((dc, dd))
            dd = np.nextafter(dd, np.float32(np.inf))
    z = np.full((3, 3 * len(pairs)), np.float32(1e30), dtype=np.float32)
    for j, (dc, dd) in enumerate(pairs):
        z[1, 3 * j + 1] = 0.0
        z[0, 3 * j + 1] = -dc
        z[0, 3 * j + 2] = -dd
    return z


def rho8_half_blocks(rnd: np.ndarray):
    """3 x 3k float32 raster of independent 3 x 3 blocks: centre 0, north
    neighbour -1, north-east neighbour -1.5, the others far higher.  With
    rho8's diagonal distance t = 2 - r the diagonal slope 1.5 / t beats the
    cardinal 1 exactly when r > 1/2.  rnd (length k) gives each block's r; the
    returned per-cell r raster puts it at the block centres (0.5 elsewhere).
    Input only: no direction is computed here."""
    k = len(rnd)
    z = np.full((3, 3 * k), np.float32(1e30), dtype=np.float32)
    r = np.full((3, 3 * k), np.float32(0.5), dtype=np.float32)
    for j in range(k):
        z[1, 3 * j + 1] = 0.0
        z[0, 3 * j + 1] = -1.0
        z[0, 3 * j + 2] = -1.5
        r[1, 3 * j + 1] = rnd[j]
    return z, r
