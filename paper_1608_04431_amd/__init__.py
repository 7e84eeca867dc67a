"""d8flow: MI355X-native D8 flow accumulation (Barnes, arXiv:1608.04431).

Thin Python binding over the C ABI of ``libd8flow.so`` (include/d8flow.h).
PyTorch provides device memory and the current stream; every step of the
computation runs in the library's HIP kernels.  Calls are asynchronous on
``torch.cuda.current_stream()``; data-dependent errors are reported by
``check_status``.
"""
from __future__ import annotations

import torch

from . import _lib
from ._lib import D8_ACC_F32, D8_ACC_U32, D8Error  # noqa: F401

NOFLOW = 8
NODATA = 9

__all__ = ["d8_directions", "d8_directions_rho8", "flow_accum", "flow_accum_adjoint", "workspace_bytes", "Workspace",
           "check_status", "FlowAccum", "FlowAccumAbsorb", "D8Error", "Raster", "Batch", "BatchGraph",
           "stream_workspace_bytes", "flow_accum_streamed", "flow_accum_absorb",
           "flow_accum_absorb_adjoint", "flow_accum_absorb_alpha_grad", "flow_accum_noalloc",
           "flow_accum_streamed_f32", "flow_accum_adjoint_streamed"]


def _stream(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else t.data_ptr()


def _check_raster(t: torch.Tensor, dtype: torch.dtype, name: str):
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 2-D tensor")


def workspace_bytes(rows: int, cols: int, tile: tuple[int, int] = (0, 0)) -> int:
    n = _lib.load().d8_workspace_bytes(rows, cols, tile[0], tile[1])
    if n == 0:
        raise D8Error(_lib.D8_EINVAL, f"tile {tile} for {rows}x{cols}")
    return n


class Workspace:
    """Caller-owned device scratch for flow_accum / flow_accum_adjoint."""

    def __init__(self, rows: int, cols: int, tile: tuple[int, int] = (0, 0), device=None,
                 also: tuple[tuple[int, int], ...] = ()):
        """Sized for `tile` and every shape in `also` (e.g. the forward's and
        the adjoint's tiles when they differ)."""
        self.rows, self.cols, self.tile = rows, cols, tuple(tile)
        self.nbytes = max(workspace_bytes(rows, cols, tuple(t)) for t in (self.tile, *also))
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device or "cuda")

    def fits(self, rows: int, cols: int, tile) -> bool:
        return workspace_bytes(rows, cols, tuple(tile)) <= self.nbytes


def _workspace(ws, rows, cols, tile, device):
    if ws is None:
        return Workspace(rows, cols, tile, device)
    return ws


def d8_directions(dem: torch.Tensor, nodata: float = -9999.0, out: torch.Tensor | None = None):
    """D8 codes (uint8) of a float32 DEM (see d8_directions in d8flow.h)."""
    _check_raster(dem, torch.float32, "dem")
    if out is None:
        out = torch.empty(dem.shape, dtype=torch.uint8, device=dem.device)
    _check_raster(out, torch.uint8, "out")
    rc = _lib.load().d8_directions(_ptr(dem), _ptr(out), dem.shape[0], dem.shape[1],
                                   float(nodata), _stream(dem.device))
    _lib.check(rc, "d8_directions")
    return out


def d8_directions_rho8(dem: torch.Tensor, rnd: torch.Tensor, nodata: float = -9999.0,
                       out: torch.Tensor | None = None):
    """rho8 codes (uint8) of a float32 DEM with one uniform draw in [0, 1) per
    cell in rnd (float32, same shape; see d8_directions_rho8 in d8flow.h)."""
    _check_raster(dem, torch.float32, "dem")
    _check_raster(rnd, torch.float32, "rnd")
    if rnd.shape != dem.shape:
        raise ValueError("rnd and dem differ in shape")
    if out is None:
        out = torch.empty(dem.shape, dtype=torch.uint8, device=dem.device)
    _check_raster(out, torch.uint8, "out")
    rc = _lib.load().d8_directions_rho8(_ptr(dem), _ptr(rnd), _ptr(out), dem.shape[0], dem.shape[1],
                                        float(nodata), _stream(dem.device))
    _lib.check(rc, "d8_directions_rho8")
    return out


def flow_accum(dirs: torch.Tensor, weights: torch.Tensor | None = None, acc_type: str = "auto",
               tile: tuple[int, int] = (0, 0), ws: Workspace | None = None,
               out: torch.Tensor | None = None, check: bool = False) -> torch.Tensor:
    """Flow accumulation A (Eq. (1)).  acc_type 'u32' (unit weights, returned
    as int32 storage holding uint32 bits) or 'f32'; 'auto' = u32 without
    weights, f32 with.  Asynchronous: data errors (an invalid code, a cycle)
    are recorded in the workspace and raised by check_status(ws), or here with
    check=True (which synchronises the stream); without either, and with no
    workspace passed, they go unreported."""
    _check_raster(dirs, torch.uint8, "dirs")
    if acc_type == "auto":
        acc_type = "u32" if weights is None else "f32"
    if acc_type not in ("u32", "f32"):
        raise ValueError("acc_type must be 'u32' or 'f32'")
    if weights is not None:
        _check_raster(weights, torch.float32, "weights")
        if weights.shape != dirs.shape:
            raise ValueError("weights and dirs differ in shape")
    rows, cols = dirs.shape
    dt = torch.int32 if acc_type == "u32" else torch.float32
    if out is None:
        out = torch.empty((rows, cols), dtype=dt, device=dirs.device)
    _check_raster(out, dt, "out")
    ws = _workspace(ws, rows, cols, tile, dirs.device)
    rc = _lib.load().flow_accum(_ptr(dirs), _ptr(weights), _ptr(out),
                                D8_ACC_U32 if acc_type == "u32" else D8_ACC_F32, rows, cols,
                                tile[0], tile[1], _ptr(ws.buf), ws.nbytes, _stream(dirs.device))
    _lib.check(rc, "flow_accum")
    if check:
        check_status(ws)
    return out


def flow_accum_noalloc(dirs: torch.Tensor, weights: torch.Tensor | None = None, acc_type: str = "auto",
                       tile: tuple[int, int] = (0, 0), out: torch.Tensor | None = None,
                       status: torch.Tensor | None = None) -> torch.Tensor:
    """flow_accum on the library's own per-GPU scratch array (no workspace, no
    device allocation in the call when `out` is given).  `status`: optional
    int32 device tensor of one element that receives the data status (0 ok,
    4 invalid code, 5 cycle).  Overlapping calls on one GPU race."""
    _check_raster(dirs, torch.uint8, "dirs")
    if acc_type == "auto":
        acc_type = "u32" if weights is None else "f32"
    if acc_type not in ("u32", "f32"):
        raise ValueError("acc_type must be 'u32' or 'f32'")
    if weights is not None:
        _check_raster(weights, torch.float32, "weights")
        if weights.shape != dirs.shape:
            raise ValueError("weights and dirs differ in shape")
    rows, cols = dirs.shape
    dt = torch.int32 if acc_type == "u32" else torch.float32
    if out is None:
        out = torch.empty((rows, cols), dtype=dt, device=dirs.device)
    _check_raster(out, dt, "out")
    if status is not None and (status.dtype != torch.int32 or not status.is_cuda or status.numel() != 1):
        raise ValueError("status must be a one-element int32 device tensor")
    rc = _lib.load().flow_accum_noalloc(_ptr(dirs), _ptr(weights), _ptr(out),
                                        D8_ACC_U32 if acc_type == "u32" else D8_ACC_F32, rows, cols,
                                        tile[0], tile[1], _ptr(status), _stream(dirs.device))
    _lib.check(rc, "flow_accum_noalloc")
    return out


def flow_accum_adjoint(dirs: torch.Tensor, grad_acc: torch.Tensor, tile=(0, 0),
                       ws: Workspace | None = None, out: torch.Tensor | None = None,
                       check: bool = False):
    """lambda = (I-P)^-T g: the sum of grad_acc along each cell's downstream
    path.  Data errors as for flow_accum (check_status(ws) or check=True)."""
    _check_raster(dirs, torch.uint8, "dirs")
    _check_raster(grad_acc, torch.float32, "grad_acc")
    if grad_acc.shape != dirs.shape:
        raise ValueError("grad_acc and dirs differ in shape")
    rows, cols = dirs.shape
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float32, device=dirs.device)
    _check_raster(out, torch.float32, "out")
    ws = _workspace(ws, rows, cols, tile, dirs.device)
    rc = _lib.load().flow_accum_adjoint(_ptr(dirs), _ptr(grad_acc), _ptr(out), rows, cols,
                                        tile[0], tile[1], _ptr(ws.buf), ws.nbytes,
                                        _stream(dirs.device))
    _lib.check(rc, "flow_accum_adjoint")
    if check:
        check_status(ws)
    return out


def flow_accum_absorb(dirs: torch.Tensor, alpha: torch.Tensor, weights: torch.Tensor | None = None,
                      tile: tuple[int, int] = (0, 0), ws: torch.Tensor | None = None,
                      out: torch.Tensor | None = None, check: bool = False) -> torch.Tensor:
    """A(p) = w(p) + sum over donors n of alpha(n) A(n), float32 (see
    flow_accum_absorb in d8flow.h).  ws: a device uint8 tensor of at least
    d8_absorb_workspace_bytes, or None.  Asynchronous; check=True synchronises
    and raises on a data error recorded in ws."""
    _check_raster(dirs, torch.uint8, "dirs")
    _check_raster(alpha, torch.float32, "alpha")
    if alpha.shape != dirs.shape:
        raise ValueError("alpha and dirs differ in shape")
    if weights is not None:
        _check_raster(weights, torch.float32, "weights")
        if weights.shape != dirs.shape:
            raise ValueError("weights and dirs differ in shape")
    rows, cols = dirs.shape
    n = _lib.load().d8_absorb_workspace_bytes(rows, cols, tile[0], tile[1])
    if n == 0:
        raise D8Error(_lib.D8_EINVAL, f"tile {tile} for {rows}x{cols}")
    if ws is None:
        ws = torch.empty(n, dtype=torch.uint8, device=dirs.device)
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float32, device=dirs.device)
    _check_raster(out, torch.float32, "out")
    rc = _lib.load().flow_accum_absorb(_ptr(dirs), _ptr(weights), _ptr(alpha), _ptr(out), rows, cols,
                                       tile[0], tile[1], _ptr(ws), ws.numel(), _stream(dirs.device))
    _lib.check(rc, "flow_accum_absorb")
    if check:
        _lib.check(_lib.load().d8_check_status(_ptr(ws), _stream(dirs.device)), "status")
    return out


def flow_accum_absorb_adjoint(dirs: torch.Tensor, alpha: torch.Tensor, grad: torch.Tensor,
                              tile: tuple[int, int] = (0, 0), ws: torch.Tensor | None = None,
                              out: torch.Tensor | None = None, check: bool = False) -> torch.Tensor:
    """lambda(c) = g(c) + alpha(c) lambda(receiver(c)), float32 (see
    flow_accum_absorb_adjoint in d8flow.h).  Asynchronous; check=True as for
    flow_accum_absorb."""
    _check_raster(dirs, torch.uint8, "dirs")
    for t, name in ((alpha, "alpha"), (grad, "grad")):
        _check_raster(t, torch.float32, name)
        if t.shape != dirs.shape:
            raise ValueError(f"{name} and dirs differ in shape")
    rows, cols = dirs.shape
    n = _lib.load().d8_absorb_workspace_bytes(rows, cols, tile[0], tile[1])
    if n == 0:
        raise D8Error(_lib.D8_EINVAL, f"tile {tile} for {rows}x{cols}")
    if ws is None:
        ws = torch.empty(n, dtype=torch.uint8, device=dirs.device)
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float32, device=dirs.device)
    _check_raster(out, torch.float32, "out")
    rc = _lib.load().flow_accum_absorb_adjoint(_ptr(dirs), _ptr(alpha), _ptr(grad), _ptr(out), rows, cols,
                                               tile[0], tile[1], _ptr(ws), ws.numel(), _stream(dirs.device))
    _lib.check(rc, "flow_accum_absorb_adjoint")
    if check:
        _lib.check(_lib.load().d8_check_status(_ptr(ws), _stream(dirs.device)), "status")
    return out


def flow_accum_absorb_alpha_grad(dirs: torch.Tensor, acc: torch.Tensor, lam: torch.Tensor,
                                 out: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dalpha(n) = A(n) lambda(receiver(n)) (see flow_accum_absorb_alpha_grad
    in d8flow.h): acc from flow_accum_absorb, lam from flow_accum_absorb_adjoint
    of dL/dA."""
    _check_raster(dirs, torch.uint8, "dirs")
    for t, name in ((acc, "acc"), (lam, "lam")):
        _check_raster(t, torch.float32, name)
        if t.shape != dirs.shape:
            raise ValueError(f"{name} and dirs differ in shape")
    if out is None:
        out = torch.empty(dirs.shape, dtype=torch.float32, device=dirs.device)
    _check_raster(out, torch.float32, "out")
    rc = _lib.load().flow_accum_absorb_alpha_grad(_ptr(dirs), _ptr(acc), _ptr(lam), _ptr(out),
                                                  dirs.shape[0], dirs.shape[1], _stream(dirs.device))
    _lib.check(rc, "flow_accum_absorb_alpha_grad")
    return out


def stream_workspace_bytes(rows: int, cols: int, tile: tuple[int, int] = (0, 0),
                           band_rows: int = 0) -> int:
    n = _lib.load().d8_stream_workspace_bytes(rows, cols, tile[0], tile[1], band_rows)
    if n == 0:
        raise D8Error(_lib.D8_EINVAL, f"tile {tile}, band_rows {band_rows} for {rows}x{cols}")
    return n


def flow_accum_streamed(dirs_host: torch.Tensor, tile: tuple[int, int] = (0, 0), band_rows: int = 0,
                        ws: torch.Tensor | None = None, out: torch.Tensor | None = None,
                        device=None, sync: bool = True) -> torch.Tensor:
    """Unit-count accumulation of a raster held in host memory, in bands of
    band_rows rows (flow_accum_streamed in d8flow.h).  dirs_host: uint8 CPU
    tensor (pinned memory lets copies overlap); returns the counts as an int32
    CPU tensor holding uint32 bits (pinned when allocated here).  With
    sync=False the result is complete once the device's current stream is,
    and `dirs_host`, `out` and `ws` must stay alive until then."""
    if dirs_host.dtype != torch.uint8 or dirs_host.is_cuda or dirs_host.dim() != 2 \
            or not dirs_host.is_contiguous():
        raise ValueError("dirs_host must be a contiguous 2-D uint8 CPU tensor")
    rows, cols = dirs_host.shape
    dev = torch.device(device or "cuda")
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.int32, pin_memory=True)
    if out.dtype != torch.int32 or out.is_cuda or tuple(out.shape) != (rows, cols) \
            or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 CPU tensor of the raster's shape")
    nbytes = stream_workspace_bytes(rows, cols, tile, band_rows)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if ws.dtype != torch.uint8 or not ws.is_cuda or ws.numel() < nbytes:
        raise ValueError(f"ws must be a device uint8 tensor of at least {nbytes} bytes")
    rc = _lib.load().flow_accum_streamed(_ptr(dirs_host), _ptr(out), rows, cols, tile[0], tile[1],
                                         band_rows, _ptr(ws), ws.numel(), _stream(ws.device))
    _lib.check(rc, "flow_accum_streamed")
    if sync:
        _lib.check(_lib.load().d8_check_status(_ptr(ws), _stream(ws.device)), "status")
    return out


def _streamed_float(fn: str, dirs_host: torch.Tensor, v_host: torch.Tensor | None, tile, band_rows, ws, out,
                    device, sync):
    if dirs_host.dtype != torch.uint8 or dirs_host.is_cuda or dirs_host.dim() != 2 \
            or not dirs_host.is_contiguous():
        raise ValueError("dirs_host must be a contiguous 2-D uint8 CPU tensor")
    rows, cols = dirs_host.shape
    if v_host is not None and (v_host.dtype != torch.float32 or v_host.is_cuda
                               or tuple(v_host.shape) != (rows, cols) or not v_host.is_contiguous()):
        raise ValueError("the float input must be a contiguous float32 CPU tensor of the raster's shape")
    dev = torch.device(device or "cuda")
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float32, pin_memory=True)
    if out.dtype != torch.float32 or out.is_cuda or tuple(out.shape) != (rows, cols) \
            or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 CPU tensor of the raster's shape")
    nbytes = stream_workspace_bytes(rows, cols, tile, band_rows)
    if ws is None:
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    if ws.dtype != torch.uint8 or not ws.is_cuda or ws.numel() < nbytes:
        raise ValueError(f"ws must be a device uint8 tensor of at least {nbytes} bytes")
    rc = getattr(_lib.load(), fn)(_ptr(dirs_host), _ptr(v_host), _ptr(out), rows, cols, tile[0], tile[1],
                                  band_rows, _ptr(ws), ws.numel(), _stream(ws.device))
    _lib.check(rc, fn)
    if sync:
        _lib.check(_lib.load().d8_check_status(_ptr(ws), _stream(ws.device)), "status")
    return out


def flow_accum_streamed_f32(dirs_host: torch.Tensor, weights_host: torch.Tensor | None = None,
                            tile: tuple[int, int] = (0, 0), band_rows: int = 0, ws: torch.Tensor | None = None,
                            out: torch.Tensor | None = None, device=None, sync: bool = True) -> torch.Tensor:
    """Float32 accumulation of a raster and its weights held in host memory
    (flow_accum_streamed_f32 in d8flow.h); returns a float32 CPU tensor
    (pinned when allocated here).  sync as for flow_accum_streamed."""
    return _streamed_float("flow_accum_streamed_f32", dirs_host, weights_host, tile, band_rows, ws, out, device,
                           sync)


def flow_accum_adjoint_streamed(dirs_host: torch.Tensor, grad_host: torch.Tensor, tile: tuple[int, int] = (0, 0),
                                band_rows: int = 0, ws: torch.Tensor | None = None,
                                out: torch.Tensor | None = None, device=None, sync: bool = True) -> torch.Tensor:
    """The adjoint of a raster held in host memory, cotangent grad_host in host
    memory (flow_accum_adjoint_streamed in d8flow.h); returns a float32 CPU
    tensor.  sync as for flow_accum_streamed."""
    if grad_host is None:
        raise ValueError("grad_host is required")
    return _streamed_float("flow_accum_adjoint_streamed", dirs_host, grad_host, tile, band_rows, ws, out, device,
                           sync)


def check_status(ws: Workspace | torch.Tensor) -> None:
    """Synchronise the current stream and raise on a data error recorded in
    ws (a Workspace or a workspace tensor)."""
    buf = ws.buf if isinstance(ws, Workspace) else ws
    rc = _lib.load().d8_check_status(_ptr(buf), _stream(buf.device))
    _lib.check(rc, "status")


def timing_enable(on: bool = True, passes_only: bool = False) -> None:
    """Bracket library kernel launches with HIP events (profiling aid): every
    launch, or with passes_only the per-tile passes alone."""
    _lib.check(_lib.load().d8_timing_enable((2 if passes_only else 1) if on else 0), "d8_timing_enable")


def timing_report(max_entries: int = 64) -> dict:
    """{kernel name: (summed ms, launches)} since the last report; waits for
    the recorded events."""
    import ctypes
    names = (ctypes.c_char_p * max_entries)()
    ms = (ctypes.c_double * max_entries)()
    cnt = (ctypes.c_int64 * max_entries)()
    n = _lib.load().d8_timing_report(names, ms, cnt, max_entries)
    if n < 0:
        raise D8Error(n, "timing_report")
    return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(n)}


class FlowAccum(torch.autograd.Function):
    """A = FlowAccum.apply(w, dirs[, tile[, tile_adj]]): differentiable in the
    weights w; the backward pass is flow_accum_adjoint, on tile_adj when given
    (the two calls need not share a tile shape)."""

    @staticmethod
    def forward(ctx, w, dirs, tile=(0, 0), tile_adj=None):
        ctx.save_for_backward(dirs)
        ctx.tile = tuple(tile)
        ctx.tile_adj = tuple(tile_adj) if tile_adj is not None else ctx.tile
        return flow_accum(dirs, w.contiguous(), acc_type="f32", tile=ctx.tile)

    @staticmethod
    def backward(ctx, grad_a):
        (dirs,) = ctx.saved_tensors
        gw = flow_accum_adjoint(dirs, grad_a.contiguous(), tile=ctx.tile_adj)
        return gw, None, None, None


class FlowAccumAbsorb(torch.autograd.Function):
    """A = FlowAccumAbsorb.apply(w, dirs, alpha[, tile]): accumulation with
    absorption, differentiable in the weights w (flow_accum_absorb_adjoint)
    and in the fractions alpha (flow_accum_absorb_alpha_grad on A and that
    adjoint)."""

    @staticmethod
    def forward(ctx, w, dirs, alpha, tile=(0, 0)):
        alpha = alpha.detach().contiguous()
        ctx.tile = tuple(tile)
        A = flow_accum_absorb(dirs, alpha, w.detach().contiguous(), tile=ctx.tile)
        ctx.save_for_backward(dirs, alpha, A)
        return A

    @staticmethod
    def backward(ctx, grad_a):
        dirs, alpha, A = ctx.saved_tensors
        lam = flow_accum_absorb_adjoint(dirs, alpha, grad_a.contiguous(), tile=ctx.tile)
        ga = flow_accum_absorb_alpha_grad(dirs, A, lam) if ctx.needs_input_grad[2] else None
        return (lam if ctx.needs_input_grad[0] else None), None, ga, None


# ----------------------------------------------------------------- batches --

class Raster:
    """One raster of a batch: dirs (uint8) and, per direction of the batch,
    weights (float32 or None) with the output acc, and grad_acc with the
    output grad_weights.  Outputs are allocated when not given."""

    def __init__(self, dirs, weights=None, grad_acc=None, tile=(0, 0), acc=None, grad_weights=None):
        _check_raster(dirs, torch.uint8, "dirs")
        for name, t in (("weights", weights), ("grad_acc", grad_acc)):
            if t is not None:
                _check_raster(t, torch.float32, name)
                if t.shape != dirs.shape:
                    raise ValueError(f"{name} and dirs differ in shape")
        self.dirs, self.weights, self.grad_acc, self.tile = dirs, weights, grad_acc, tuple(tile)
        self.acc = acc if acc is not None else torch.empty(dirs.shape, dtype=torch.float32,
                                                           device=dirs.device)
        self.grad_weights = grad_weights
        if grad_acc is not None and grad_weights is None:
            self.grad_weights = torch.empty(dirs.shape, dtype=torch.float32, device=dirs.device)

    def item(self) -> _lib.BatchItem:
        return _lib.BatchItem(_ptr(self.dirs), _ptr(self.weights), _ptr(self.acc),
                              _ptr(self.grad_acc), _ptr(self.grad_weights), self.dirs.shape[0],
                              self.dirs.shape[1], self.tile[0], self.tile[1])


class Batch:
    """Many rasters through one set of launches (flow_accum_batched).
    mode: 'fwd', 'adj' or 'fwd+adj'."""

    def __init__(self, rasters: list[Raster], mode: str = "fwd+adj", device=None):
        self.rasters = list(rasters)
        self.mode = {"fwd": _lib.D8_BATCH_FWD, "adj": _lib.D8_BATCH_ADJ,
                     "fwd+adj": _lib.D8_BATCH_FWD | _lib.D8_BATCH_ADJ}[mode]
        self.items = (_lib.BatchItem * max(1, len(self.rasters)))(*[r.item() for r in self.rasters])
        self.n = len(self.rasters)
        self.nbytes = _lib.load().d8_batch_workspace_bytes(self.items, self.n)
        if self.nbytes == 0:
            raise D8Error(_lib.D8_EINVAL, "batch items")
        dev = device or (self.rasters[0].dirs.device if self.rasters else "cuda")
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)

    def run(self) -> None:
        rc = _lib.load().flow_accum_batched(self.items, self.n, self.mode, _ptr(self.buf),
                                            self.nbytes, _stream(self.buf.device))
        _lib.check(rc, "flow_accum_batched")

    def check_status(self) -> None:
        rc = _lib.load().d8_check_status(_ptr(self.buf), _stream(self.buf.device))
        _lib.check(rc, "status")

    def graph(self) -> "BatchGraph":
        return BatchGraph(self)


class BatchGraph:
    """The batch recorded as one HIP graph (d8_graph_create); launch() replays
    it on the current stream."""

    def __init__(self, batch: Batch):
        import ctypes
        self.batch = batch
        h = ctypes.c_void_p()
        rc = _lib.load().d8_graph_create(batch.items, batch.n, batch.mode, _ptr(batch.buf),
                                         batch.nbytes, _stream(batch.buf.device), ctypes.byref(h))
        _lib.check(rc, "d8_graph_create")
        self.handle = h

    def launch(self) -> None:
        if self.handle is None:
            raise RuntimeError("graph destroyed")
        rc = _lib.load().d8_graph_launch(self.handle, _stream(self.batch.buf.device))
        _lib.check(rc, "d8_graph_launch")

    def destroy(self) -> None:
        if self.handle is not None:
            _lib.load().d8_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
