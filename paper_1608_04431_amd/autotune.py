"""Tile-shape autotuner.

Times candidate tile shapes on a sample raster of a size class (forward in
float32 and the adjoint, each on its own, events on the current stream) and
keeps the fastest per (device, size class) in a JSON cache: one shape for
both calls ("tile") and the fastest for each call ("tile_fwd", "tile_adj");
the two calls need not share a shape.  The paper leaves the tile
size free (Section "The Algorithm": equal tiles are a convenience); on the GPU
it trades LDS per tile (resident tiles per CU) against the number of
perimeter cells in the global graph.

Cache lookup order: the user cache (``$D8_TUNE_CACHE`` or
``~/.cache/d8flow/tiles.json``), then the table shipped with the package
(``tiles_mi355x.json``), then 64 x 64.
"""
from __future__ import annotations

import json
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
PACKAGED = os.path.join(HERE, "tiles_mi355x.json")
DEFAULT_TILE = (64, 64)
CANDIDATES = ((64, 64), (64, 44), (64, 40), (64, 32), (32, 64), (64, 48), (48, 64), (32, 32))


def size_class(rows: int, cols: int) -> str:
    """Rasters are grouped by their longer side, rounded up to a power of two
    (at least 64)."""
    s = max(int(rows), int(cols), 1)
    k = max(6, (s - 1).bit_length())
    return str(1 << k)


def device_key(device=None) -> str:
    if not torch.cuda.is_available():
        return "cpu"
    props = torch.cuda.get_device_properties(device or torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "") or ""
    return f"{props.name}|{arch.split(':')[0]}"


def user_cache_path() -> str:
    return os.environ.get("D8_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "d8flow", "tiles.json")


def _read(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


class Tuner:
    """tile_for(rows, cols) -> (tile_rows, tile_cols); tune(...) measures."""

    def __init__(self, path: str | None = None, device=None):
        self.path = path or user_cache_path()
        self.device = device
        self.key = device_key(device)
        self.user = _read(self.path)
        self.packaged = _read(PACKAGED)

    def _key(self, batch: bool) -> str:
        return self.key + ("|batch" if batch else "")

    def lookup(self, rows: int, cols: int, batch: bool = False, kind: str | None = None):
        """The cached tile for the size class: this device's entry, else one
        for its architecture (the packaged table is keyed by architecture),
        else the entry of the nearest tuned class.
        kind "fwd" / "adj" takes that call's own shape where one is stored."""
        cls = size_class(rows, cols)
        arch = self.key.split("|")[-1]
        keys = (self._key(batch), arch + ("|batch" if batch else ""))
        tables = [table.get(key, {}) for table in (self.user, self.packaged) for key in keys]
        entry = next((t[cls] for t in tables if t.get(cls)), None)
        if entry is None:
            # no entry for the class: the nearest tuned class (in powers of
            # two; the larger on a tie), the user's cache first
            near = [(abs(int(c).bit_length() - int(cls).bit_length()), -int(c), i, e)
                    for i, t in enumerate(tables) for c, e in t.items() if e]
            if not near:
                return None
            entry = min(near, key=lambda x: x[:3])[3]
        t = entry.get(f"tile_{kind}") if kind else None
        return tuple(int(v) for v in (t or entry["tile"]))

    def tile_for(self, rows: int, cols: int, batch: bool = False, kind: str | None = None) -> tuple[int, int]:
        """Tile shape for a raster run on its own, or (batch=True) as one of
        many rasters in a batch (a batch lookup falls back to the single one);
        kind "fwd" or "adj" for the forward or the adjoint call alone."""
        if batch:
            t = self.lookup(rows, cols, True)
            if t:
                return t
        return self.lookup(rows, cols, kind=kind) or DEFAULT_TILE

    def tune(self, dirs: torch.Tensor, weights: torch.Tensor | None = None,
             grad_acc: torch.Tensor | None = None, candidates=CANDIDATES, reps: int = 3,
             save: bool = True) -> dict:
        """Times forward (float32) + adjoint for every candidate on `dirs`
        (a sample of its size class), records the fastest for the class and
        returns {tile: ms}."""
        from . import Workspace, flow_accum, flow_accum_adjoint
        rows, cols = dirs.shape
        if weights is None:
            weights = torch.ones(dirs.shape, dtype=torch.float32, device=dirs.device)
        if grad_acc is None:
            grad_acc = torch.ones(dirs.shape, dtype=torch.float32, device=dirs.device)
        acc = torch.empty(dirs.shape, dtype=torch.float32, device=dirs.device)
        lam = torch.empty_like(acc)
        fwd, adj = {}, {}
        for tile in candidates:
            th, tw = min(tile[0], rows), min(tile[1], cols)
            if (th, tw) in fwd:
                continue
            ws = Workspace(rows, cols, (th, tw), dirs.device)
            for out, call in ((fwd, lambda: flow_accum(dirs, weights, "f32", (th, tw), ws, acc)),
                              (adj, lambda: flow_accum_adjoint(dirs, grad_acc, (th, tw), ws, lam))):
                call()
                start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                best = None
                for _ in range(reps):
                    start.record()
                    call()
                    stop.record()
                    stop.synchronize()
                    ms = start.elapsed_time(stop)
                    best = ms if best is None else min(best, ms)
                out[(th, tw)] = best
        times = {t: fwd[t] + adj[t] for t in fwd}
        tile = min(times, key=times.get)
        tf, ta = min(fwd, key=fwd.get), min(adj, key=adj.get)
        cls = size_class(rows, cols)
        self.user.setdefault(self.key, {})[cls] = {
            "tile": list(tile), "ms": round(times[tile], 4), "sample": [rows, cols],
            "tile_fwd": list(tf), "tile_adj": list(ta), "ms_split": round(fwd[tf] + adj[ta], 4),
            "candidates": {f"{a}x{b}": round(v, 4) for (a, b), v in times.items()},
            "candidates_fwd": {f"{a}x{b}": round(v, 4) for (a, b), v in fwd.items()},
            "candidates_adj": {f"{a}x{b}": round(v, 4) for (a, b), v in adj.items()}}
        if save:
            self.save()
        return times

    def tune_batch(self, samples, candidates=CANDIDATES, reps: int = 2, save: bool = True) -> dict:
        """Tile shape for rasters of one size class run together: times one
        recorded batch (forward float32 + adjoint) of all `samples` -- a
        list of (dirs, weights, grad_acc) -- per candidate.  In a batch the
        other rasters supply the parallelism, so this favours per-cell
        efficiency where tune() favours one raster's latency."""
        from . import Batch, Raster
        if not samples:
            return {}
        outs = [(torch.empty_like(w), torch.empty_like(g)) for _, w, g in samples]
        cls = size_class(*max((d.shape for d, _, _ in samples), key=lambda s: s[0] * s[1]))
        times = {}
        for tile in candidates:
            rasters = [Raster(d, w, g, tile=tile, acc=a, grad_weights=l)
                       for (d, w, g), (a, l) in zip(samples, outs)]
            graph = Batch(rasters, "fwd+adj", samples[0][0].device).graph()
            try:
                graph.launch()
                start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                best = None
                for _ in range(reps):
                    start.record()
                    graph.launch()
                    stop.record()
                    stop.synchronize()
                    ms = start.elapsed_time(stop)
                    best = ms if best is None else min(best, ms)
            finally:
                graph.destroy()
            times[tuple(tile)] = best
        tile = min(times, key=times.get)
        self.user.setdefault(self._key(True), {})[cls] = {
            "tile": list(tile), "ms": round(times[tile], 4), "rasters": len(samples),
            "candidates": {f"{a}x{b}": round(v, 4) for (a, b), v in times.items()}}
        if save:
            self.save()
        return times

    def save(self) -> None:
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.user, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def table_from_bench(bench: dict, arch: str) -> dict:
    """A packaged table from one bench.py JSON line: the batch leg's tunings
    (per size class, one raster and batch context) and the main workload's
    tile sweep (its size class, one raster)."""
    b = bench.get("batched") or {}
    single, batch = {}, {}
    for src, dst in ((b.get("tuning_single_ms", {}), single), (b.get("tuning_ms", {}), batch)):
        for cls, cands in src.items():
            best = min(cands, key=cands.get)
            dst[cls] = {"tile": [int(v) for v in best.split("x")], "ms": cands[best],
                        "candidates": cands}
    sweep = bench.get("tile_sweep_ms_per_step") or {}
    if sweep:
        rows, cols = bench["config"]["rows"], bench["config"]["cols"]
        best = min(sweep, key=sweep.get)
        entry = {"tile": [int(v) for v in best.split("x")], "ms": sweep[best], "candidates": sweep}
        for kind in ("fwd", "adj"):
            split = bench.get(f"tile_sweep_ms_{kind}") or {}
            if split:
                b = min(split, key=split.get)
                entry[f"tile_{kind}"] = [int(v) for v in b.split("x")]
                entry[f"candidates_{kind}"] = split
        single[size_class(rows, cols)] = entry
    return {arch: single, arch + "|batch": batch}


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="write a tile table from a bench.py JSON line")
    ap.add_argument("bench_json")
    ap.add_argument("--arch", default="gfx950")
    ap.add_argument("--out", default=PACKAGED)
    a = ap.parse_args()
    with open(a.bench_json) as f:
        line = [ln for ln in f if ln.strip().startswith("{")][-1]
    table = table_from_bench(json.loads(line), a.arch)
    table["source"] = f"bench.py tuning legs ({os.path.basename(a.bench_json)})"
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(a.out)
