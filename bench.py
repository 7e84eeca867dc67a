"""Benchmark: D8 flow accumulation, forward (unit weights, uint32) plus adjoint
(dense float32 cotangent), on a 32768 x 32768 synthetic raster, one GPU.

One step = flow_accum + flow_accum_adjoint over the whole raster, inputs
resident in HBM.  Prints one JSON line (see the keys below).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import tempfile
import time
from multiprocessing import shared_memory

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "D8 accumulation cells/s (fwd+adjoint) at 32768², % HBM peak; batched vs looped"
HBM_PEAK_GBPS = 8000.0

# Algorithmic bytes per cell of each tile kernel: its share of what the step
# must move at minimum (forward: read codes, write A; adjoint: read codes and
# g, write lambda).  Re-reads (the second pass reads the codes again), the
# adjoint's retained lambda_loc and root labels, and the per-perimeter-cell
# records are not counted.
KERNEL_BYTES_PER_CELL = {
    "fwd_pass1": 1.0,   # directions
    "fwd_pass2": 4.0,   # uint32 A
    "adj_pass1": 5.0,   # directions + g
    "adj_pass2": 4.0,   # lambda
    "d8_directions": 5.0,
    "d8_directions_rho8": 9.0,  # z 4 + r 4 + code 1
    "flow_accum_absorb": 13.0,  # code 1 + alpha 4 + w 4 read, A 4 written
    "flow_accum_absorb_adjoint": 13.0,  # code 1 + alpha 4 + g 4 read, lambda 4 written
}
STEP_BYTES_PER_CELL = 14.0  # forward 1 + 4, adjoint 1 + 4 + 4
SWEEP_TILES = ((64, 64), (64, 48), (64, 44), (64, 40), (64, 36), (64, 32), (64, 28), (60, 32), (56, 32),
               (56, 48), (48, 48), (48, 32))


ABSORB_TILE = (48, 32)  # the absorption entry points' default shape

KERNEL_NAMES = {  # timing label -> kernel symbol prefix in profiler output
    "fwd_pass1": "fwd_walk<1, unsigned int",
    "fwd_pass2": "fwd_walk<2, unsigned int",
    "adj_pass1": "adj_walk",
    "adj_pass2": "adj_finish",
}
SOURCES = ("paper_1608_04431_amd/csrc/d8flow.hip", "paper_1608_04431_amd/csrc/kernels.h",
           "paper_1608_04431_amd/csrc/walk.h", "paper_1608_04431_amd/csrc/d8_common.h")


def source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<kernel>_<workload>.txt), or None when there is none or
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_sha():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


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
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n / (t2 - t0), "unit": "cells/s", "cores": 1, "kind": "oracle",
            "host_cpu": model, "host_threads": os.cpu_count(),
            "sample": f"rows 0..{rows - 1} of the {z.shape[0]}x{z.shape[1]} raster "
                      f"({n} cells): Kahn forward in uint64 ({t1 - t0:.2f}s) + reverse-order "
                      f"adjoint in float64 ({t2 - t1:.2f}s), serial C"}


def cpu_oracle_configs() -> dict:
    """The CPU oracle (serial C, one thread) on the two smaller workloads,
    whole rasters: dem512 (unit counts) and dem8192_ocean (unit counts, then
    float64 sums of the float32 weights of seed 21).  D8 is not timed."""
    import oracle
    out = {}
    for name in ("dem512", "dem8192_ocean"):
        wl = synth.WORKLOADS[name]
        d = oracle.d8(synth.workload_dem(name))
        t0 = time.perf_counter()
        oracle.accum_u64(d)
        t1 = time.perf_counter()
        rec = {"cells": int(d.size), "u32_cells_per_s": d.size / (t1 - t0), "cores": 1, "kind": "oracle"}
        if "seed_w" in wl:
            w = synth.uniform(d.shape, wl["seed_w"])
            t2 = time.perf_counter()
            oracle.accum_f64(d, w)
            rec["f32_weighted_cells_per_s"] = d.size / (time.perf_counter() - t2)
        out[name] = rec
    return out


# ------------------------------------------------------------ batched leg --
# 2000 DEMs of uneven sizes (side log-uniform in [64, 4096], aspect uniform in
# [0.5, 2]), float32 weights and cotangents: forward + adjoint for all of
# them as one recorded graph launch, against a loop of per-DEM calls.

_SHM = {}


def _batch_worker_init(names):
    os.environ["OMP_NUM_THREADS"] = "1"
    for k, name in names.items():
        _SHM[k] = shared_memory.SharedMemory(name=name)


def _batch_worker(job):
    off, rows, cols, lam, sd, sw, sg = job
    n = rows * cols
    for key, arr in (("dem", synth.dem(rows, cols, seed=sd, lambda0=lam)),
                     ("w", synth.uniform((rows, cols), sw)), ("g", synth.uniform((rows, cols), sg))):
        dst = np.ndarray((n,), dtype=np.float32, buffer=_SHM[key].buf, offset=4 * off)
        dst[:] = arr.ravel()
    return n


class BatchData:
    """DEMs, weights and cotangents of the batch in shared memory."""

    def __init__(self, n: int, workers: int):
        self.shapes = synth.batch_shapes(n)
        self.off = np.concatenate([[0], np.cumsum([r * c for r, c, *_ in self.shapes])]).astype(np.int64)
        total = int(self.off[-1])
        self.shm = {k: shared_memory.SharedMemory(create=True, size=max(4, 4 * total))
                    for k in ("dem", "w", "g")}
        try:
            jobs = [(int(self.off[i]), *self.shapes[i][:3], *self.shapes[i][3:])
                    for i in range(n)]
            jobs.sort(key=lambda j: -(j[1] * j[2]))
            names = {k: v.name for k, v in self.shm.items()}
            with mp.get_context("fork").Pool(workers, _batch_worker_init, (names,)) as pool:
                done = sum(pool.imap_unordered(_batch_worker, jobs, chunksize=4))
            assert done == total
        except BaseException:
            self.close()
            raise
        self.cells = total

    def view(self, key: str, i: int) -> np.ndarray:
        rows, cols = self.shapes[i][:2]
        return np.ndarray((rows, cols), dtype=np.float32, buffer=self.shm[key].buf,
                          offset=4 * int(self.off[i]))

    def close(self):
        for v in self.shm.values():
            try:
                v.close()
                v.unlink()
            except FileNotFoundError:
                pass
        self.shm = {}


def _oracle_worker(job):
    """One DEM of the batch through the CPU oracle: D8 (not timed), then the
    Kahn forward in float64 and the reverse-order adjoint, timed."""
    import oracle
    i, rows, cols, off = job
    n = rows * cols
    view = lambda key: np.ndarray((rows, cols), dtype=np.float32, buffer=_SHM[key].buf, offset=4 * off)
    d = oracle.d8(view("dem"))
    w, g = view("w"), view("g")
    t0 = time.perf_counter()
    _, order = oracle.accum_f64(d, w, want_order=True)
    oracle.transpose_f64(d, g, order)
    return n, time.perf_counter() - t0


def oracle_batch_baseline(bd: BatchData, workers: int, max_cells: float = 1.5e9) -> dict | None:
    """The CPU oracle over the batch's first DEMs (up to max_cells cells), one
    DEM per task on `workers` host processes (the paper's delegation of tiles
    to workers): aggregate cells/s = the sum over processes of their cells
    over their summed accumulate + adjoint time.  Runs before anything
    touches the GPU."""
    jobs, cells = [], 0
    for i, (rows, cols, *_rest) in enumerate(bd.shapes):
        if cells >= max_cells:
            break
        jobs.append((i, rows, cols, int(bd.off[i])))
        cells += rows * cols
    jobs.sort(key=lambda j: -(j[1] * j[2]))
    names = {k: v.name for k, v in bd.shm.items()}
    per_worker = {}
    with mp.get_context("fork").Pool(workers, _batch_worker_init, (names,)) as pool:
        for (n, t), pid in pool.imap_unordered(_oracle_worker_pid, jobs, chunksize=1):
            c, tt = per_worker.get(pid, (0, 0.0))
            per_worker[pid] = (c + n, tt + t)
    slowest = max(tt for _, tt in per_worker.values())
    rate = sum(c / tt for c, tt in per_worker.values() if tt > 0)
    return {"value": rate, "unit": "cells/s", "cores": len(per_worker), "kind": "oracle",
            "sample": f"the first {len(jobs)} of the batch's {len(bd.shapes)} DEMs ({cells} cells): float64 "
                      f"Kahn forward + reverse-order adjoint per DEM (D8 not timed), one DEM per task on "
                      f"{workers} host processes; value = the sum of the processes' own rates; "
                      f"slowest process {slowest:.2f}s ({cells / slowest:.3e} cells/s by it)"}


def _oracle_worker_pid(job):
    return _oracle_worker(job), os.getpid()


def batch_leg(bd: BatchData, reps: int) -> dict:
    import torch
    import paper_1608_04431_amd as d8
    from paper_1608_04431_amd.autotune import Tuner, size_class
    dev = torch.device("cuda:0")
    n = len(bd.shapes)
    rs = []
    for i in range(n):
        dem = torch.from_numpy(bd.view("dem", i)).to(dev)
        dirs = d8.d8_directions(dem)
        del dem
        rs.append(dict(dirs=dirs, w=torch.from_numpy(bd.view("w", i)).to(dev),
                       g=torch.from_numpy(bd.view("g", i)).to(dev)))
    torch.cuda.synchronize()
    bd.close()
    log(f"batch resident: {n} DEMs, {bd.cells:.3e} cells")

    # tile shape per size class, tuned in batch context on the class's DEMs
    with tempfile.TemporaryDirectory() as tmp:
        tuner = Tuner(path=os.path.join(tmp, "tiles.json"))
        classes = {}
        for r in rs:
            classes.setdefault(size_class(*r["dirs"].shape), []).append(r)
        tuned = {}
        for cls, members in sorted(classes.items(), key=lambda kv: int(kv[0])):
            times = tuner.tune_batch([(r["dirs"], r["w"], r["g"]) for r in members], save=False)
            tuned[cls] = {f"{a}x{b}": round(v, 4) for (a, b), v in times.items()}
        tuned_single = {}
        for cls, members in sorted(classes.items(), key=lambda kv: int(kv[0])):
            big = max(members, key=lambda r: r["dirs"].numel())
            times = tuner.tune(big["dirs"], big["w"], big["g"], reps=2, save=False)
            tuned_single[cls] = {f"{a}x{b}": round(v, 4) for (a, b), v in times.items()}
        for r in rs:
            r["tile"] = tuner.tile_for(*r["dirs"].shape, batch=True)
            r["tile1"] = tuner.tile_for(*r["dirs"].shape)
    choice = {cls: "x".join(map(str, tuner.tile_for(int(cls), int(cls), batch=True))) for cls in tuned}
    choice1 = {cls: "x".join(map(str, tuner.tile_for(int(cls), int(cls)))) for cls in tuned}
    log(f"tiles per size class: batch {choice}, single {choice1}")

    # (i) looped: two C-ABI calls per DEM on one stream, one sync at the end
    ws_bytes = max(max(d8.workspace_bytes(*r["dirs"].shape, r["tile"]),
                       d8.workspace_bytes(*r["dirs"].shape, r["tile1"])) for r in rs)
    ws = d8.Workspace(1, 1, (1, 1), dev)
    ws.buf = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    ws.nbytes = ws_bytes
    for r in rs:
        r["acc"] = torch.empty_like(r["w"])
        r["gw"] = torch.empty_like(r["w"])

    def looped(key="tile"):
        for r in rs:
            d8.flow_accum(r["dirs"], r["w"], "f32", r[key], ws, r["acc"])
            d8.flow_accum_adjoint(r["dirs"], r["g"], r[key], ws, r["gw"])

    def timed(fn):
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        out = []
        for _ in range(reps):
            torch.cuda.synchronize()
            start.record()
            fn()
            stop.record()
            torch.cuda.synchronize()
            out.append(start.elapsed_time(stop))
        return float(np.median(out)), out

    looped()
    torch.cuda.synchronize()
    d8.timing_enable(True)
    looped()
    torch.cuda.synchronize()
    d8.timing_enable(False)
    launches_looped = sum(c for _, c in d8.timing_report().values())
    looped("tile1")
    t_loop1, _ = timed(lambda: looped("tile1"))
    t_loop, loop_all = timed(looped)
    d8.check_status(ws)
    log(f"looped: {t_loop:.2f} ms with the batch tiles, {t_loop1:.2f} ms with per-raster tiles "
        f"(medians of {reps})")

    # (ii) batched: one graph launch for all DEMs, forward + adjoint
    rasters = [d8.Raster(r["dirs"], r["w"], r["g"], tile=r["tile"]) for r in rs]
    batch = d8.Batch(rasters, "fwd+adj", dev)
    # per-kernel times of the same work, launched without the graph
    batch.run()
    torch.cuda.synchronize()
    d8.timing_enable(True)
    batch.run()
    torch.cuda.synchronize()
    d8.timing_enable(False)
    batch_kernels = {k: round(ms, 3) for k, (ms, c) in d8.timing_report().items()}
    graph = batch.graph()
    try:
        graph.launch()
        t_graph, graph_all = timed(graph.launch)
        batch.check_status()
    finally:
        graph.destroy()
    log(f"batched graph: {t_graph:.2f} ms (median of {reps})")
    same = all(torch.equal(rr.acc, r["acc"]) and torch.equal(rr.grad_weights, r["gw"])
               for rr, r in zip(rasters, rs))
    bytes_alg = 18.0 * bd.cells  # forward 1 + 4 + 4, adjoint 1 + 4 + 4 bytes per cell
    return {
        "workload": f"{n} DEMs, sides log-uniform in [64, 4096], aspect uniform in [0.5, 2], "
                    "filled value-noise terrain (wavelength max side / 8), float32 weights and "
                    "cotangents U[0,1); forward (f32) + adjoint",
        "dems": n, "cells": int(bd.cells),
        "looped_ms": t_loop, "batched_ms": t_graph, "speedup": t_loop / t_graph,
        "looped_per_raster_tiles_ms": t_loop1, "speedup_vs_per_raster_tiles": t_loop1 / t_graph,
        "looped_cells_per_s": bd.cells / (t_loop * 1e-3),
        "batched_cells_per_s": bd.cells / (t_graph * 1e-3),
        "batched_hbm_GBps_algorithmic": bytes_alg / (t_graph * 1e-3) / 1e9,
        "batched_frac_hbm_peak": bytes_alg / (t_graph * 1e-3) / 1e9 / HBM_PEAK_GBPS,
        "launches_looped": int(launches_looped), "launches_batched": 1,
        "reps_ms": {"looped": [round(x, 3) for x in loop_all], "batched": [round(x, 3) for x in graph_all]},
        "tiles": choice, "tiles_per_raster": choice1, "tuning_ms": tuned,
        "tuning_single_ms": tuned_single, "outputs_identical": bool(same),
        "kernels_ms": batch_kernels,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="dem32768")
    ap.add_argument("--tile", type=int, nargs=2, default=None,
                    help="tile shape of both calls of the timed run (default: the autotuner's "
                         "table, which holds one shape per call)")
    ap.add_argument("--no-sweep", action="store_true", help="skip the tile-shape sweep")
    ap.add_argument("--cache-dir", default=os.environ.get("D8_CACHE_DIR"))
    ap.add_argument("--cpu-rows", type=int, default=6144,
                    help="rows of the raster in the CPU-oracle sample (0 = skip)")
    ap.add_argument("--batch", type=int, default=2000,
                    help="DEMs in the batched-vs-looped leg (0 = skip)")
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="host processes generating the batch")
    ap.add_argument("--stream-band", type=int, default=0, metavar="ROWS",
                    help="rows per band of the streamed leg (0 = the library's default)")
    ap.add_argument("--no-stream", action="store_true",
                    help="skip the streamed leg (raster in pinned host memory)")
    ap.add_argument("--no-absorb", action="store_true",
                    help="skip the timing of accumulation with absorption")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of MIB MiB before timing (a kernel of known "
                         "traffic for scaling hardware counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(row bands of tiles per GPU with one exchange of band-boundary records "
              "would shard it; not built).", file=sys.stderr)
        sys.exit(2)

    # the batch is generated by forked workers before anything touches the GPU
    bd = None
    if args.batch > 0:
        t = time.time()
        bd = BatchData(args.batch, args.workers)
        log(f"generated batch of {args.batch} DEMs ({bd.cells:.3e} cells) in {time.time() - t:.1f}s "
            f"with {args.workers} workers")
    cpu_batch = None
    if bd is not None and args.cpu_rows > 0:
        # the oracle on all host workers, before anything touches the GPU
        try:
            cpu_batch = oracle_batch_baseline(bd, args.workers)
            log(f"oracle over the batch: {cpu_batch['value']:.3e} cells/s on {cpu_batch['cores']} processes")
        except Exception as e:  # reported, never fatal to the bench line
            cpu_batch = {"error": repr(e)}
    try:
        out = run(args, bd)
        if cpu_batch is not None and out.get("batched") is not None:
            out["batched"]["cpu_baseline"] = cpu_batch
    finally:
        if bd is not None:
            bd.close()
    print(json.dumps(out), flush=True)


def absorb_leg(d8, dirs, w, tile, seed, reps=3):
    """Eq. (1) with absorption and its adjoint on the same directions:
    alpha ~ U[0.5, 1) per cell, the adjoint's U[0, 1) draws as weights and as
    g; events around `reps` calls after one warm call, on the launch stream."""
    import torch
    rows, cols = dirs.shape
    alpha = torch.from_numpy(0.5 + 0.5 * synth.uniform((rows, cols), seed)).to(dirs.device)
    ws = torch.empty(d8._lib.load().d8_absorb_workspace_bytes(rows, cols, *tile), dtype=torch.uint8,
                     device=dirs.device)
    out = torch.empty((rows, cols), dtype=torch.float32, device=dirs.device)
    lam = torch.empty_like(out)
    res = {"alpha": "U[0.5,1) per cell", "weights and g": "U[0,1)", "tile": list(tile)}
    for name, fn in (("flow_accum_absorb", lambda: d8.flow_accum_absorb(dirs, alpha, w, tile=tile, ws=ws,
                                                                        out=out)),
                     ("flow_accum_absorb_adjoint", lambda: d8.flow_accum_absorb_adjoint(
                         dirs, alpha, w, tile=tile, ws=ws, out=lam))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        gbps = KERNEL_BYTES_PER_CELL[name] * rows * cols / (ms * 1e-3) / 1e9
        log(f"{name}: {ms:.3f} ms, {gbps:.0f} GB/s algorithmic")
        res[name] = {"ms": round(ms, 4), "cells_per_s": rows * cols / (ms * 1e-3),
                     "bytes_per_cell": KERNEL_BYTES_PER_CELL[name], "achieved_GBps": gbps,
                     "frac_hbm_peak": gbps / HBM_PEAK_GBPS}
    del alpha, ws, out, lam
    torch.cuda.empty_cache()
    return res


def streamed_leg(d8, dirs, A, g, lam, tile, tile_a, band_rows, reps=3):
    """The raster in pinned host memory, streamed in bands: the unit-count
    forward (flow_accum_streamed), the float32 forward with weights in host
    memory (flow_accum_streamed_f32; the cotangent's U[0, 1) values serve as
    weights) and the adjoint (flow_accum_adjoint_streamed, the same dense
    cotangent), each timed with events around the whole call (host copies
    included) and compared with the in-memory results."""
    import torch
    rows, cols = dirs.shape
    cells = rows * cols
    dirs_h = dirs.cpu().pin_memory()
    g_h = g.cpu().pin_memory()
    nbytes = max(d8.stream_workspace_bytes(rows, cols, t, band_rows) for t in (tile, tile_a))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dirs.device)

    def timed(call, out):
        call(out, True)
        times = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            call(out, False)
            e1.record()
            e1.synchronize()
            times.append(e0.elapsed_time(e1))
        d8._lib.check(d8._lib.load().d8_check_status(ws.data_ptr(), torch.cuda.current_stream().cuda_stream),
                      "status")
        return sorted(times)[len(times) // 2]

    out_u = torch.empty((rows, cols), dtype=torch.int32, pin_memory=True)
    ms_u = timed(lambda o, sync: d8.flow_accum_streamed(dirs_h, tile=tile, band_rows=band_rows, ws=ws, out=o,
                                                         sync=sync), out_u)
    same_u = bool(torch.equal(out_u, A.cpu()))
    del out_u
    out_f = torch.empty((rows, cols), dtype=torch.float32, pin_memory=True)
    ms_f = timed(lambda o, sync: d8.flow_accum_streamed_f32(dirs_h, g_h, tile=tile, band_rows=band_rows, ws=ws,
                                                             out=o, sync=sync), out_f)
    ref_f = d8.flow_accum(dirs, g, acc_type="f32", tile=tile).cpu()
    same_f = bool(torch.equal(out_f, ref_f))
    del out_f, ref_f
    out_a = torch.empty((rows, cols), dtype=torch.float32, pin_memory=True)
    ms_a = timed(lambda o, sync: d8.flow_accum_adjoint_streamed(dirs_h, g_h, tile=tile_a, band_rows=band_rows,
                                                                 ws=ws, out=o, sync=sync), out_a)
    lam_h = lam.cpu()
    rel_a = float(((out_a.double() - lam_h.double()).abs() / lam_h.double().abs().clamp_min(1e-30)).max())
    del out_a, lam_h
    th = min(tile[0], rows)
    band = band_rows or 16 * th
    log(f"streamed (host-resident raster): u32 fwd {ms_u:.2f} ms (identical: {same_u}), f32 fwd {ms_f:.2f} ms "
        f"(identical: {same_f}), adjoint {ms_a:.2f} ms (max rel diff to in-memory {rel_a:.2e})")

    def rec(ms, hb):
        return {"ms": round(ms, 3), "cells_per_s": cells / (ms * 1e-3), "host_bytes_per_cell": hb,
                "host_link_GBps": hb * cells / (ms * 1e-3) / 1e9}
    return {"band_rows": band, "workspace_GiB": round(nbytes / 2**30, 3),
            "u32_forward": dict(rec(ms_u, 6), outputs_identical=same_u),
            "f32_forward": dict(rec(ms_f, 14), outputs_identical=same_f),
            "adjoint": dict(rec(ms_a, 14), max_rel_diff_in_memory=rel_a),
            "what": "the forward (u32 counts; f32 with host weights) and the adjoint of the same raster from "
                    "pinned host memory: codes copied twice, a float input twice (f32, adjoint) and the "
                    "result once; median of 3, copies included"}


def run(args, bd):
    import torch
    import paper_1608_04431_amd as d8

    wl = synth.WORKLOADS[args.workload]
    z = load_dem(args.workload, args.cache_dir)
    rows, cols = z.shape
    n_cells = rows * cols
    dev = torch.device("cuda:0")
    from paper_1608_04431_amd.autotune import Tuner
    tuner = Tuner()
    tile_f = tuple(args.tile) if args.tile else tuner.tile_for(rows, cols, kind="fwd")
    tile_a = tuple(args.tile) if args.tile else tuner.tile_for(rows, cols, kind="adj")
    tile = tile_f  # the forward's shape also serves the streamed leg

    # inputs resident in HBM before timing
    dem = torch.from_numpy(z).to(dev)
    dirs = d8.d8_directions(dem)
    # D8 directions on their own (not part of the step): events around 5 runs
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        d8.d8_directions(dem, out=dirs)
    e1.record()
    torch.cuda.synchronize()
    d8_ms = e0.elapsed_time(e1) / 5
    d8_gbps = KERNEL_BYTES_PER_CELL["d8_directions"] * n_cells / (d8_ms * 1e-3) / 1e9
    log(f"d8_directions: {d8_ms:.3f} ms, {d8_gbps:.0f} GB/s algorithmic")
    # rho8 on the same DEM, one U[0,1) draw per cell (an input)
    gen = torch.Generator(device=dev)
    gen.manual_seed(8)
    rnd = torch.rand((rows, cols), generator=gen, device=dev, dtype=torch.float32)
    dr8 = d8.d8_directions_rho8(dem, rnd)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(5):
        d8.d8_directions_rho8(dem, rnd, out=dr8)
    e1.record()
    torch.cuda.synchronize()
    rho8_ms = e0.elapsed_time(e1) / 5
    rho8_gbps = KERNEL_BYTES_PER_CELL["d8_directions_rho8"] * n_cells / (rho8_ms * 1e-3) / 1e9
    log(f"d8_directions_rho8: {rho8_ms:.3f} ms, {rho8_gbps:.0f} GB/s algorithmic")
    del dem, rnd, dr8
    g = torch.from_numpy(synth.uniform((rows, cols), wl.get("seed_g", 31))).to(dev)
    A = torch.empty((rows, cols), dtype=torch.int32, device=dev)
    lam = torch.empty((rows, cols), dtype=torch.float32, device=dev)

    # tile-shape sweep: each call on its own, 3 runs per candidate after a
    # warm one (the timed run below uses the autotuner's choices, or --tile)
    sweep, sweep_f, sweep_a = {}, {}, {}
    if not args.no_sweep:
        for cand in SWEEP_TILES:
            wsc = d8.Workspace(rows, cols, cand, dev)
            key = f"{cand[0]}x{cand[1]}"
            for out, call in ((sweep_f, lambda: d8.flow_accum(dirs, acc_type="u32", tile=cand, ws=wsc, out=A)),
                              (sweep_a, lambda: d8.flow_accum_adjoint(dirs, g, tile=cand, ws=wsc, out=lam))):
                call()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(3):
                    call()
                e1.record()
                torch.cuda.synchronize()
                out[key] = round(e0.elapsed_time(e1) / 3, 3)
            d8.check_status(wsc)
            sweep[key] = round(sweep_f[key] + sweep_a[key], 3)
            del wsc
        log(f"tile sweep (ms): forward {sweep_f}, adjoint {sweep_a}")
    ws = d8.Workspace(rows, cols, tile_f, dev, also=(tile_a,))
    if args.calibrate_copy > 0:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst
    # achievable HBM bandwidth on this device: a plain 4 GiB device copy
    # (bytes read + written over the copy's time, best of 3)
    src = torch.empty(1 << 30, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms = []
    for _ in range(3):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        copy_ms.append(e0.elapsed_time(e1))
    copy_gbps = 2 * src.numel() * 4 / (min(copy_ms) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    log(f"device copy: {copy_gbps:.0f} GB/s (read + write)")
    torch.cuda.synchronize()
    log(f"inputs resident: {rows}x{cols}, tiles {tile_f} (forward) and {tile_a} (adjoint), "
        f"workspace {ws.nbytes / 2**30:.2f} GiB")

    def step():
        d8.flow_accum(dirs, acc_type="u32", tile=tile_f, ws=ws, out=A)
        d8.flow_accum_adjoint(dirs, g, tile=tile_a, ws=ws, out=lam)

    for _ in range(args.warmup):
        step()
    d8.check_status(ws)
    torch.cuda.synchronize()
    log("warmup done")

    # per-kernel events only around the tile passes here (the dominant kernel
    # is one of them); the full breakdown comes from separate steps below
    d8.timing_enable(True, passes_only=True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    # events between the two calls of every step (no synchronisation inside)
    marks = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps + 1)]
    torch.cuda.synchronize()
    start.record()
    marks[0].record()
    for i in range(args.steps):
        d8.flow_accum(dirs, acc_type="u32", tile=tile_f, ws=ws, out=A)
        marks[2 * i + 1].record()
        d8.flow_accum_adjoint(dirs, g, tile=tile_a, ws=ws, out=lam)
        marks[2 * i + 2].record()
    stop.record()
    torch.cuda.synchronize()
    d8.timing_enable(False)
    ms_total = start.elapsed_time(stop)
    t_fwd = [marks[2 * i].elapsed_time(marks[2 * i + 1]) for i in range(args.steps)]
    t_adj = [marks[2 * i + 1].elapsed_time(marks[2 * i + 2]) for i in range(args.steps)]
    t_step = [a + b for a, b in zip(t_fwd, t_adj)]
    kernels = d8.timing_report()
    d8.check_status(ws)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step")
    # every kernel, over a few more steps (events around all launches add
    # about 2 % to a step, so these steps are not the timed ones)
    n_break = min(args.steps, 3)
    d8.timing_enable(True)
    for _ in range(n_break):
        step()
    torch.cuda.synchronize()
    d8.timing_enable(False)
    breakdown = d8.timing_report()

    # dominant kernel: the one with the largest share of the step
    per_launch = {k: (ms / n, n / args.steps) for k, (ms, n) in kernels.items()}
    dom = max(kernels, key=lambda k: kernels[k][0])
    dom_tile = tile_a if dom.startswith("adj") else tile_f
    dom_ms = per_launch[dom][0]
    dom_bytes = KERNEL_BYTES_PER_CELL.get(dom)
    roofline = {"bound": "hbm", "kernel": dom, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "traffic": measured_traffic(dom, f"{args.workload}_{dom_tile[0]}x{dom_tile[1]}")}
    if dom_bytes is not None:
        achieved = dom_bytes * n_cells / (dom_ms * 1e-3) / 1e9
        roofline.update(achieved=achieved, frac=achieved / HBM_PEAK_GBPS,
                        bytes_per_launch=dom_bytes * n_cells, avg_launch_ms=dom_ms)
    else:
        roofline.update(achieved=None, frac=None, avg_launch_ms=dom_ms,
                        note="latency-bound graph kernel: no per-cell byte model")
    step_gbps = STEP_BYTES_PER_CELL * n_cells / (ms_step * 1e-3) / 1e9

    absorb = None
    if not args.no_absorb:
        absorb = absorb_leg(d8, dirs, g, ABSORB_TILE, wl.get("seed_g", 31) + 1)

    streamed = None
    if not args.no_stream:
        streamed = streamed_leg(d8, dirs, A, g, lam, tile_f, tile_a, args.stream_band)

    cpu = None
    if args.cpu_rows > 0:
        log("timing the CPU oracle sample")
        cpu = cpu_baseline(z, wl.get("seed_g", 31), min(args.cpu_rows, rows))
        cpu["other_workloads"] = cpu_oracle_configs()

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
                   "cells": n_cells, "rows": rows, "cols": cols, "tile_fwd": list(tile_f),
                   "tile_adj": list(tile_a),
                   "parallelism": "single GPU"},
        "ms_per_step_median": float(np.median(t_step)),
        "ms_per_step_min": float(np.min(t_step)),
        "t_fwd_ms_median": float(np.median(t_fwd)),
        "t_adj_ms_median": float(np.median(t_adj)),
        "hbm_copy_GBps": copy_gbps,
        "step_hbm_GBps_algorithmic": step_gbps,
        "step_frac_hbm_peak": step_gbps / HBM_PEAK_GBPS,
        "kernels_ms_per_step": {k: round(ms / n_break, 4) for k, (ms, n) in breakdown.items()},
        "passes_ms_per_step_timed": {k: round(ms / args.steps, 4) for k, (ms, n) in kernels.items()},
        "tile_sweep_ms_per_step": sweep,
        "tile_sweep_ms_fwd": sweep_f,
        "tile_sweep_ms_adj": sweep_a,
        "tuner_device_key": __import__("paper_1608_04431_amd.autotune", fromlist=["x"]).device_key(),
        "roofline": roofline,
        "d8_directions": {"ms": round(d8_ms, 4), "bytes_per_cell": KERNEL_BYTES_PER_CELL["d8_directions"],
                          "achieved_GBps": d8_gbps, "frac_hbm_peak": d8_gbps / HBM_PEAK_GBPS},
        "d8_directions_rho8": {"ms": round(rho8_ms, 4),
                               "bytes_per_cell": KERNEL_BYTES_PER_CELL["d8_directions_rho8"],
                               "achieved_GBps": rho8_gbps, "frac_hbm_peak": rho8_gbps / HBM_PEAK_GBPS},
        "absorb": absorb,
        "streamed": streamed,
        "cpu_baseline": cpu,
    }
    if bd is not None:
        del A, lam, ws, dirs, g
        torch.cuda.empty_cache()
        out["batched"] = batch_leg(bd, args.batch_reps)
    return out


if __name__ == "__main__":
    main()
