"""Benchmark: D8 flow accumulation, forward (unit weights, uint32) plus adjoint
(dense float32 cotangent), on a 32768 x 32768 synthetic raster, one GPU.

One step = flow_accum + flow_accum_adjoint over the whole raster, inputs
resident in HBM.  Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "D8 accumulation cells/s (fwd+adjoint) at 32768², % HBM peak; batched vs looped"
HBM_PEAK_GBPS = 8000.0

# Algorithmic bytes per cell of each tile kernel (what the operation must read
# and write at minimum; records and workspace traffic are not counted).
KERNEL_BYTES_PER_CELL = {
    "fwd_pass1": 1.0,   # directions
    "fwd_pass2": 5.0,   # directions + uint32 A
    "adj_pass1": 5.0,   # directions + g
    "adj_pass2": 9.0,   # directions + g + lambda
    "d8_directions": 5.0,
}
STEP_BYTES_PER_CELL = 14.0  # forward 1 + 4, adjoint 1 + 4 + 4


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_dem(name: str, cache_dir: str | None) -> np.ndarray:
    w = synth.WORKLOADS[name]
    path = os.path.join(cache_dir, f"{name}_dem.npy") if cache_dir else None
    if path and os.path.exists(path):
        log(f"loading cached DEM {path}")
        return np.load(path, mmap_mode=None)
    t = time.time()
    z = synth.workload_dem(name)
    log(f"generated DEM {name} {z.shape} in {time.time() - t:.1f}s")
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        np.save(path, z)
    return z


def cpu_baseline(z: np.ndarray, seed_g: int, rows: int) -> dict:
    """The CPU oracle (serial C, one thread) on a band of the same raster:
    forward in uint64 plus the float64 transpose solve."""
    import oracle
    band = np.ascontiguousarray(z[:rows])
    d = oracle.d8(band)
    g = synth.uniform(band.shape, seed_g)
    t0 = time.perf_counter()
    _, order = oracle.accum_u64(d, want_order=True)
    t1 = time.perf_counter()
    oracle.transpose_f64(d, g, order)
    t2 = time.perf_counter()
    n = band.size
    return {"value": n / (t2 - t0), "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"rows 0..{rows - 1} of the {z.shape[0]}x{z.shape[1]} raster "
                      f"({n} cells): Kahn forward in uint64 ({t1 - t0:.2f}s) + reverse-order "
                      f"adjoint in float64 ({t2 - t1:.2f}s), serial C"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dem32768")
    ap.add_argument("--tile", type=int, nargs=2, default=(64, 64))
    ap.add_argument("--cache-dir", default=os.environ.get("D8_CACHE_DIR"))
    ap.add_argument("--cpu-rows", type=int, default=6144,
                    help="rows of the raster in the CPU-oracle sample (0 = skip)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the method would shard).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1608_04431_amd as d8

    wl = synth.WORKLOADS[args.workload]
    z = load_dem(args.workload, args.cache_dir)
    rows, cols = z.shape
    n_cells = rows * cols
    dev = torch.device("cuda:0")
    tile = tuple(args.tile)

    # inputs resident in HBM before timing
    dem = torch.from_numpy(z).to(dev)
    dirs = d8.d8_directions(dem)
    del dem
    g = torch.from_numpy(synth.uniform((rows, cols), wl.get("seed_g", 31))).to(dev)
    A = torch.empty((rows, cols), dtype=torch.int32, device=dev)
    lam = torch.empty((rows, cols), dtype=torch.float32, device=dev)
    ws = d8.Workspace(rows, cols, tile, dev)
    torch.cuda.synchronize()
    log(f"inputs resident: {rows}x{cols}, tile {tile}, workspace {ws.nbytes / 2**30:.2f} GiB")

    def step():
        d8.flow_accum(dirs, acc_type="u32", tile=tile, ws=ws, out=A)
        d8.flow_accum_adjoint(dirs, g, tile=tile, ws=ws, out=lam)

    for _ in range(args.warmup):
        step()
    d8.check_status(ws)
    torch.cuda.synchronize()
    log("warmup done")

    d8.timing_enable(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    d8.timing_enable(False)
    ms_total = start.elapsed_time(stop)
    kernels = d8.timing_report()
    d8.check_status(ws)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step")

    # dominant kernel: the one with the largest share of the step
    per_launch = {k: (ms / n, n / args.steps) for k, (ms, n) in kernels.items()}
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_ms = per_launch[dom][0]
    dom_bytes = KERNEL_BYTES_PER_CELL.get(dom)
    roofline = {"bound": "hbm", "kernel": dom, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "traffic": None}
    if dom_bytes is not None:
        achieved = dom_bytes * n_cells / (dom_ms * 1e-3) / 1e9
        roofline.update(achieved=achieved, frac=achieved / HBM_PEAK_GBPS,
                        bytes_per_launch=dom_bytes * n_cells, avg_launch_ms=dom_ms)
    else:
        roofline.update(achieved=None, frac=None, avg_launch_ms=dom_ms,
                        note="latency-bound graph kernel: no per-cell byte model")
    step_gbps = STEP_BYTES_PER_CELL * n_cells / (ms_step * 1e-3) / 1e9

    cpu = None
    if args.cpu_rows > 0:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(z, wl.get("seed_g", 31), min(args.cpu_rows, rows))

    out = {
        "metric": METRIC,
        "value": n_cells / (ms_step * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 fwd / f32 adj",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {rows}x{cols} uint8 D8 directions of a filled "
                               f"6-octave value-noise DEM (wavelength {wl['lambda0']}), unit "
                               f"weights uint32 forward + dense U[0,1) float32 adjoint",
                   "cells": n_cells, "tile": list(tile), "parallelism": "single GPU"},
        "step_hbm_GBps_algorithmic": step_gbps,
        "step_frac_hbm_peak": step_gbps / HBM_PEAK_GBPS,
        "kernels_ms_per_step": {k: round(ms / args.steps, 4) for k, (ms, n) in kernels.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
