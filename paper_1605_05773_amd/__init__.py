"""D8 flow directions and up-slope area on MI355X (gfx950).

Thin Python binding over the C ABI in include/d8.h (libd8.so, built in-tree by
build_lib.py).  Every step of the computation runs in the library's HIP
kernels; this module only marshals arguments: PyTorch supplies device memory
(the caching allocator) and the current HIP stream.  There is no CPU fallback:
if libd8.so is missing every call raises.

    dirs = flowdirs(dem)                       # uint8 codes, same shape
    A = accum(dirs)                            # uint32 counts (Eq. 1, w = 1)
    A = accum(dirs, weights)                   # float32 weighted
    A = D8Accum.apply(dirs, weights)           # differentiable in weights
    g = accum_backward(dirs, grad_out)         # adjoint
"""
from __future__ import annotations

import ctypes
import json
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libd8.so")

D8_OK, D8_EINVAL, D8_ENOMEM, D8_EHIP, D8_EBADDIR, D8_ECYCLE, D8_EUNSUPPORTED = range(7)
D8_U32, D8_F32 = 0, 1
NONE, NODATA = 8, 255

_lib = None


class D8Error(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        msg = _lib.d8_strerror(status).decode() if _lib is not None else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)
        self.status = status


class d8_desc(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32)]


def lib():
    """The loaded libd8.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        sig = {
            "d8_flowdirs": ([P, I64, I64, P, P], I32),
            "d8_flowdirs_steepest": ([P, I64, I64, P, P], I32),
            "d8_workspace_bytes": ([I64, I64, I32], SZ),
            "d8_backward_workspace_bytes": ([I64, I64, I32], SZ),
            "d8_accum": ([P, I64, I64, P, I32, P, P, P, SZ, I32, P], I32),
            "d8_accum_noalloc": ([P, I64, I64, P, I32, P, P, I32, P, P], I32),
            "d8_accum_backward": ([P, I64, I64, P, P, P, SZ, I32, P], I32),
            "d8_accum_dem": ([P, I64, I64, P, P, P, SZ, I32, P], I32),
            "d8_accum_streamed_workspace_bytes": ([I64, I64, I64], SZ),
            "d8_accum_streamed": ([P, I64, I64, P, I64, P, SZ, P], I32),
            "d8_fill_workspace_bytes": ([I64, I64], SZ),
            "d8_fill_eps": ([P, I64, I64, ctypes.c_float, P, P, SZ, P, P], I32),
            "d8_batched_workspace_bytes": ([P, I32, I32], SZ),
            "d8_batched_backward_workspace_bytes": ([P, I32, I32], SZ),
            "d8_flowdirs_batched": ([P, P, P, I32, P, P, SZ, P], I32),
            "d8_accum_batched": ([P, P, P, I32, P, I32, P, P, P, SZ, I32, I32, P], I32),
            "d8_accum_backward_batched": ([P, P, P, I32, P, P, P, SZ, I32, I32, P], I32),
            "d8_autotune_batched": ([P, P, P, I32, P, P, P, P, SZ, P, P, P, P], I32),
            "d8_device_status": ([P, P, P], I32),
            "d8_phase_timing": ([I32], I32),
            "d8_phase_report": ([I32, P, P, P], I32),
            "d8_strerror": ([I32], ctypes.c_char_p),
            "d8_version": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


EXPORTED = (
    "d8_flowdirs", "d8_flowdirs_steepest", "d8_workspace_bytes", "d8_accum", "d8_accum_dem", "d8_accum_backward",
    "d8_batched_workspace_bytes", "d8_flowdirs_batched", "d8_accum_batched", "d8_accum_backward_batched", "d8_autotune_batched",
    "d8_device_status", "d8_strerror", "d8_version", "d8_phase_timing", "d8_phase_report",
    "d8_fill_workspace_bytes", "d8_fill_eps", "d8_accum_streamed_workspace_bytes", "d8_accum_streamed",
    "d8_accum_noalloc", "d8_backward_workspace_bytes", "d8_batched_backward_workspace_bytes",
)
NPHASES = 10


def _check(st: int, what: str):
    if st != D8_OK:
        raise D8Error(st, what)


def _stream(dev: torch.device) -> int:
    return torch.cuda.current_stream(dev).cuda_stream


def _dev_tensor(t: torch.Tensor, dtype, name: str):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name}: expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    return t


_ws_cache: dict = {}


def workspace(nbytes: int, device) -> torch.Tensor:
    """A cached device workspace of at least nbytes (256-byte aligned)."""
    device = torch.device(device)
    key = device.index if device.index is not None else torch.cuda.current_device()
    cur = _ws_cache.get(key)
    if cur is None or cur.numel() < nbytes + 256:
        cur = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        _ws_cache[key] = cur
    base = cur.data_ptr()
    pad = (-base) % 256
    return cur[pad:pad + nbytes]


def flowdirs(dem: torch.Tensor, rule: str = "lowest") -> torch.Tensor:
    """D8 codes of a float32 DEM (NaN = NoData): rule "lowest" (lowest of
    eight) or "steepest" (largest drop over distance, diagonals at sqrt 2)."""
    dem = _dev_tensor(dem, torch.float32, "dem")
    if dem.dim() != 2:
        raise ValueError("dem must be 2-D")
    fn = {"lowest": "d8_flowdirs", "steepest": "d8_flowdirs_steepest"}.get(rule)
    if fn is None:
        raise ValueError(f"unknown rule {rule!r}")
    out = torch.empty(dem.shape, dtype=torch.uint8, device=dem.device)
    _check(getattr(lib(), fn)(dem.data_ptr(), dem.shape[0], dem.shape[1], out.data_ptr(), _stream(dem.device)), fn)
    return out


def workspace_bytes(rows: int, cols: int, tile: int = 0, backward: bool = False) -> int:
    """Workspace bytes of the forward calls, or of the backward (backward=True)."""
    f = lib().d8_backward_workspace_bytes if backward else lib().d8_workspace_bytes
    n = f(rows, cols, tile)
    if n == 0:
        raise D8Error(D8_EINVAL, "d8_backward_workspace_bytes" if backward else "d8_workspace_bytes")
    return n


def accum(dirs: torch.Tensor, weights: torch.Tensor | None = None, *, tile: int = 0, out: torch.Tensor | None = None,
          out_lo: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Up-slope area of every cell (Eq. 1): uint32 counts, or float32 if weighted."""
    dirs = _dev_tensor(dirs, torch.uint8, "dirs")
    H, W = dirs.shape
    if weights is None and out_lo is None and (out is None or out.dtype == torch.uint32):
        dt = D8_U32
        if out is None:
            out = torch.empty((H, W), dtype=torch.uint32, device=dirs.device)
    else:
        dt = D8_F32
        if weights is not None:
            weights = _dev_tensor(weights, torch.float32, "weights")
            if weights.shape != dirs.shape:
                raise ValueError("weights shape")
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=dirs.device)
    if out_lo is not None:
        _dev_tensor(out_lo, torch.float32, "out_lo")
    nb = workspace_bytes(H, W, tile)
    if ws is None:
        ws = workspace(nb, dirs.device)
    _check(lib().d8_accum(dirs.data_ptr(), H, W, None if weights is None else weights.data_ptr(), dt,
                          out.data_ptr(), None if out_lo is None else out_lo.data_ptr(), ws.data_ptr(), ws.numel(),
                          tile, _stream(dirs.device)), "d8_accum")
    _maybe_debug_check(ws, dirs.device)
    return out


def accum_noalloc(dirs: torch.Tensor, weights: torch.Tensor | None = None, *, out: torch.Tensor,
                  out_lo: torch.Tensor | None = None, tile: int = 0, status: torch.Tensor | None = None) -> torch.Tensor:
    """accum() for callers that cannot allocate: the library's static device
    scratch replaces the workspace and nothing is allocated, so `out` (and
    `status`, a device int32/uint32 tensor of one element that receives the
    data-error word) must be given.  Raises D8Error(D8_ENOMEM) for shapes the
    scratch cannot hold."""
    dirs = _dev_tensor(dirs, torch.uint8, "dirs")
    H, W = dirs.shape
    if out.dtype == torch.uint32:
        dt = D8_U32
    else:
        dt = D8_F32
        _dev_tensor(out, torch.float32, "out")
    if weights is not None:
        weights = _dev_tensor(weights, torch.float32, "weights")
    if out.shape != dirs.shape or (weights is not None and weights.shape != dirs.shape):
        raise ValueError("shape mismatch")
    if out_lo is not None:
        _dev_tensor(out_lo, torch.float32, "out_lo")
    st = None
    if status is not None:
        if not status.is_cuda or status.numel() < 1 or status.element_size() != 4:
            raise TypeError("status: expected a device tensor of one 32-bit element")
        st = status.data_ptr()
    _check(lib().d8_accum_noalloc(dirs.data_ptr(), H, W, None if weights is None else weights.data_ptr(), dt,
                                  out.data_ptr(), None if out_lo is None else out_lo.data_ptr(), tile, st,
                                  _stream(dirs.device)), "d8_accum_noalloc")
    return out


def accum_dem(dem: torch.Tensor, *, tile: int = 0, out: torch.Tensor | None = None,
              dirs: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Fused flow directions + counts of a float32 DEM: returns (counts uint32,
    dirs uint8), equal to accum(flowdirs(dem))."""
    dem = _dev_tensor(dem, torch.float32, "dem")
    if dem.dim() != 2:
        raise ValueError("dem must be 2-D")
    H, W = dem.shape
    out = torch.empty((H, W), dtype=torch.uint32, device=dem.device) if out is None else out
    dirs = torch.empty((H, W), dtype=torch.uint8, device=dem.device) if dirs is None else dirs
    nb = workspace_bytes(H, W, tile)
    ws = workspace(nb, dem.device) if ws is None else ws
    _check(lib().d8_accum_dem(dem.data_ptr(), H, W, dirs.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(), tile,
                              _stream(dem.device)), "d8_accum_dem")
    return out, dirs


def accum_streamed(dirs_host: torch.Tensor, *, strip_rows: int = 4096, out: torch.Tensor | None = None,
                   device=None, ws: torch.Tensor | None = None) -> torch.Tensor:
    """Up-slope counts of a direction field held in host memory (a CPU uint8
    tensor, pinned for full PCIe rate): row strips of strip_rows rows (a
    multiple of 64) stream through the GPU twice.  Returns uint32 counts in
    host memory (pinned when allocated here).  Synchronises the stream."""
    if not isinstance(dirs_host, torch.Tensor) or dirs_host.is_cuda or dirs_host.dtype != torch.uint8:
        raise TypeError("dirs_host: expected a CPU uint8 tensor")
    if dirs_host.dim() != 2 or not dirs_host.is_contiguous():
        raise ValueError("dirs_host must be 2-D and contiguous")
    H, W = dirs_host.shape
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint32, pin_memory=dirs_host.is_pinned())
    elif out.is_cuda or out.dtype != torch.uint32 or out.shape != dirs_host.shape or not out.is_contiguous():
        raise TypeError("out: expected a contiguous CPU uint32 tensor of the same shape")
    nb = lib().d8_accum_streamed_workspace_bytes(H, W, strip_rows)
    if nb == 0:
        raise D8Error(D8_EINVAL, "d8_accum_streamed_workspace_bytes")
    ws = workspace(nb, dev) if ws is None else ws
    _check(lib().d8_accum_streamed(dirs_host.data_ptr(), H, W, out.data_ptr(), strip_rows, ws.data_ptr(), ws.numel(),
                                   _stream(dev)), "d8_accum_streamed")
    return out


def fill(dem: torch.Tensor, eps: float = 1e-3, *, out: torch.Tensor | None = None,
         ws: torch.Tensor | None = None, return_rounds: bool = False):
    """Epsilon-filled copy of a float32 DEM (NaN = NoData): pits and flats
    raised so that lowest-of-eight drains every cell to the DEM boundary or
    to NoData.  Synchronises the current stream.  With return_rounds, returns
    (filled, number of tile rounds that had work)."""
    dem = _dev_tensor(dem, torch.float32, "dem")
    if dem.dim() != 2:
        raise ValueError("dem must be 2-D")
    H, W = dem.shape
    out = torch.empty((H, W), dtype=torch.float32, device=dem.device) if out is None else out
    _dev_tensor(out, torch.float32, "out")
    nb = lib().d8_fill_workspace_bytes(H, W)
    if nb == 0:
        raise D8Error(D8_EINVAL, "d8_fill_workspace_bytes")
    ws = workspace(nb, dem.device) if ws is None else ws
    rounds = ctypes.c_int64(0)
    _check(lib().d8_fill_eps(dem.data_ptr(), H, W, ctypes.c_float(eps), out.data_ptr(), ws.data_ptr(), ws.numel(),
                             ctypes.byref(rounds), _stream(dem.device)), "d8_fill_eps")
    return (out, rounds.value) if return_rounds else out


def accum_backward(dirs: torch.Tensor, grad_out: torch.Tensor, *, tile: int = 0,
                   ws: torch.Tensor | None = None) -> torch.Tensor:
    """Gradient of a loss w.r.t. the weights given dL/dA: sums of grad_out along
    each cell's downstream path."""
    dirs = _dev_tensor(dirs, torch.uint8, "dirs")
    grad_out = _dev_tensor(grad_out, torch.float32, "grad_out")
    H, W = dirs.shape
    gw = torch.empty((H, W), dtype=torch.float32, device=dirs.device)
    nb = workspace_bytes(H, W, tile, backward=True)
    if ws is None:
        ws = workspace(nb, dirs.device)
    _check(lib().d8_accum_backward(dirs.data_ptr(), H, W, grad_out.data_ptr(), gw.data_ptr(), ws.data_ptr(),
                                   ws.numel(), tile, _stream(dirs.device)), "d8_accum_backward")
    _maybe_debug_check(ws, dirs.device)
    return gw


def device_status(ws: torch.Tensor | None = None, device=None) -> int:
    """Synchronises and returns the device status of the last call on ws
    (D8_OK, D8_EBADDIR or D8_ECYCLE)."""
    if ws is None:
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        ws = _ws_cache[dev.index if dev.index is not None else torch.cuda.current_device()]
        base = ws.data_ptr()
        ws = ws[(-base) % 256:]
    st = ctypes.c_int32(0)
    _check(lib().d8_device_status(ws.data_ptr(), _stream(ws.device), ctypes.byref(st)), "d8_device_status")
    return st.value


def phase_timing(enable: bool):
    """Start (clearing totals) or stop per-phase HIP-event timing in the library."""
    _check(lib().d8_phase_timing(1 if enable else 0), "d8_phase_timing")


def phase_report() -> dict:
    """{phase name: (total ms, timed calls)} for every phase timed since phase_timing(True)."""
    out = {}
    for i in range(NPHASES):
        name = ctypes.c_char_p()
        ms = ctypes.c_float(0)
        n = ctypes.c_int32(0)
        _check(lib().d8_phase_report(i, ctypes.byref(name), ctypes.byref(ms), ctypes.byref(n)), "d8_phase_report")
        if n.value:
            out[name.value.decode()] = (ms.value, n.value)
    return out


def _maybe_debug_check(ws, device):
    if os.environ.get("D8_DEBUG") == "1":
        st = device_status(ws)
        if st != D8_OK:
            raise D8Error(st, "device")


class D8Accum(torch.autograd.Function):
    """Weighted up-slope area, differentiable in the weights.

    forward(dirs, w) -> A (float32); backward(dL/dA) -> dL/dw through the
    adjoint kernel (no gradient for dirs)."""

    @staticmethod
    def forward(ctx, dirs, weights, tile: int = 0):
        ctx.save_for_backward(dirs)
        ctx.tile = tile
        return accum(dirs, weights.contiguous(), tile=tile)

    @staticmethod
    def backward(ctx, grad_out):
        (dirs,) = ctx.saved_tensors
        gw = accum_backward(dirs, grad_out.contiguous().to(torch.float32), tile=ctx.tile)
        return None, gw, None


# ------------------------------------------------------------------ batched --

class Batch:
    """n DEMs of uneven shapes packed into one device buffer."""

    def __init__(self, shapes, device):
        self.shapes = [(int(r), int(c)) for r, c in shapes]
        self.device = torch.device(device)
        offs, o = [], 0
        for r, c in self.shapes:
            offs.append(o)
            o += r * c
        self.offsets = offs
        self.total = o
        self.n = len(self.shapes)
        self.host_desc = (d8_desc * self.n)(*[d8_desc(off, r, c) for off, (r, c) in zip(offs, self.shapes)])
        raw = torch.frombuffer(bytearray(ctypes.string_at(ctypes.addressof(self.host_desc),
                                                          ctypes.sizeof(self.host_desc))), dtype=torch.uint8)
        self.dev_desc = raw.to(self.device)

    def pack(self, arrays, dtype):
        out = torch.empty(self.total, dtype=dtype, device=self.device)
        for off, (r, c), a in zip(self.offsets, self.shapes, arrays):
            out[off:off + r * c].copy_(torch.as_tensor(a).reshape(-1).to(dtype), non_blocking=False)
        return out

    def unpack(self, packed):
        return [packed[off:off + r * c].view(r, c) for off, (r, c) in zip(self.offsets, self.shapes)]

    def workspace_bytes(self, tile=0, backward=False):
        """Workspace bytes of the batched forward calls, or of the backward."""
        f = lib().d8_batched_backward_workspace_bytes if backward else lib().d8_batched_workspace_bytes
        n = f(ctypes.addressof(self.host_desc), self.n, tile)
        if n == 0:
            raise D8Error(D8_EINVAL, "d8_batched_workspace_bytes")
        return n


def flowdirs_batched(batch: Batch, dem_packed: torch.Tensor, ws=None) -> torch.Tensor:
    dem_packed = _dev_tensor(dem_packed, torch.float32, "dem_packed")
    out = torch.empty(batch.total, dtype=torch.uint8, device=batch.device)
    nb = batch.workspace_bytes(0)
    ws = workspace(nb, batch.device) if ws is None else ws
    _check(lib().d8_flowdirs_batched(dem_packed.data_ptr(), ctypes.addressof(batch.host_desc),
                                     batch.dev_desc.data_ptr(), batch.n, out.data_ptr(), ws.data_ptr(), ws.numel(),
                                     _stream(batch.device)), "d8_flowdirs_batched")
    return out


def accum_batched(batch: Batch, dirs_packed, w_packed=None, *, tile=0, waves=0, out=None, out_lo=None, ws=None):
    dirs_packed = _dev_tensor(dirs_packed, torch.uint8, "dirs_packed")
    if w_packed is None and out_lo is None and (out is None or out.dtype == torch.uint32):
        dt = D8_U32
        out = torch.empty(batch.total, dtype=torch.uint32, device=batch.device) if out is None else out
    else:
        dt = D8_F32
        out = torch.empty(batch.total, dtype=torch.float32, device=batch.device) if out is None else out
    nb = batch.workspace_bytes(tile)
    ws = workspace(nb, batch.device) if ws is None else ws
    _check(lib().d8_accum_batched(dirs_packed.data_ptr(), ctypes.addressof(batch.host_desc),
                                  batch.dev_desc.data_ptr(), batch.n,
                                  None if w_packed is None else w_packed.data_ptr(), dt, out.data_ptr(),
                                  None if out_lo is None else out_lo.data_ptr(), ws.data_ptr(), ws.numel(), tile,
                                  waves, _stream(batch.device)), "d8_accum_batched")
    return out


def accum_backward_batched(batch: Batch, dirs_packed, g_packed, *, tile=0, waves=0, out=None, ws=None):
    dirs_packed = _dev_tensor(dirs_packed, torch.uint8, "dirs_packed")
    g_packed = _dev_tensor(g_packed, torch.float32, "g_packed")
    out = torch.empty(batch.total, dtype=torch.float32, device=batch.device) if out is None else out
    nb = batch.workspace_bytes(tile, backward=True)
    ws = workspace(nb, batch.device) if ws is None else ws
    _check(lib().d8_accum_backward_batched(dirs_packed.data_ptr(), ctypes.addressof(batch.host_desc),
                                           batch.dev_desc.data_ptr(), batch.n, g_packed.data_ptr(), out.data_ptr(),
                                           ws.data_ptr(), ws.numel(), tile, waves, _stream(batch.device)),
           "d8_accum_backward_batched")
    return out


# ---------------------------------------------------------------- autotune --

def _bucket(batch: Batch) -> str:
    """Size bucket of a batch: DEM count, total cells and longest side, each
    rounded to a power of two."""
    def p2(x):
        return 1 << max(0, int(x - 1).bit_length())
    side = max(max(r, c) for r, c in batch.shapes)
    return f"n{p2(batch.n)}_cells{p2(batch.total)}_side{p2(side)}"


def autotune_batched(batch: Batch, dirs_packed, w_packed, *, cache_path=None):
    """Fastest (tile, waves) of the batched forward+backward on these inputs.

    Runs d8_autotune_batched (it synchronises the stream) unless cache_path
    (a JSON file) already holds a result for the batch's size bucket; new
    results are written back.  Returns (tile, waves, ms)."""
    key = _bucket(batch)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            e = cache[key]
            return int(e["tile"]), int(e["waves"]), float(e["ms"])
    dirs_packed = _dev_tensor(dirs_packed, torch.uint8, "dirs_packed")
    w_packed = _dev_tensor(w_packed, torch.float32, "w_packed")
    out = torch.empty(batch.total, dtype=torch.float32, device=batch.device)
    g = torch.empty(batch.total, dtype=torch.float32, device=batch.device)
    ws = workspace(batch.workspace_bytes(32, backward=True), batch.device)
    bt, bw, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0)
    _check(lib().d8_autotune_batched(dirs_packed.data_ptr(), ctypes.addressof(batch.host_desc),
                                     batch.dev_desc.data_ptr(), batch.n, w_packed.data_ptr(), out.data_ptr(),
                                     g.data_ptr(), ws.data_ptr(), ws.numel(), ctypes.byref(bt), ctypes.byref(bw),
                                     ctypes.byref(ms), _stream(batch.device)), "d8_autotune_batched")
    res = (bt.value, bw.value, ms.value)
    if cache_path:
        cache[key] = {"tile": res[0], "waves": res[1], "ms": res[2]}
        tmp = f"{cache_path}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return res


# ----------------------------------------------------------- graph launch --

class BatchedGraph:
    """The batched weighted forward and its backward captured once as a HIP
    graph (torch.cuda.CUDAGraph is a HIP graph under ROCm) over fixed device
    buffers; replay() re-runs both on whatever the input buffers hold.

    Every library call only enqueues kernels on the current stream (no
    allocation, synchronisation or memset), so the sequence is capturable.
    Inputs: the `dirs`, `w` and `g` tensors (packed, fixed addresses) —
    overwrite them in place between replays.  Outputs: `area` and `grad`."""

    def __init__(self, batch: Batch, *, tile=0, waves=0):
        self.batch = batch
        dev = batch.device
        n = batch.total
        self.dirs = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.w = torch.zeros(n, dtype=torch.float32, device=dev)
        self.g = torch.zeros(n, dtype=torch.float32, device=dev)
        self.area = torch.zeros(n, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(n, dtype=torch.float32, device=dev)
        nb = batch.workspace_bytes(tile, backward=True)  # serves the forward too
        raw = torch.empty(nb + 256, dtype=torch.uint8, device=dev)
        pad = (-raw.data_ptr()) % 256
        self._raw = raw
        self.ws = raw[pad:pad + nb]
        self.tile, self.waves = tile, waves
        self.graph = None

    def _enqueue(self):
        accum_batched(self.batch, self.dirs, self.w, tile=self.tile, waves=self.waves, out=self.area, ws=self.ws)
        accum_backward_batched(self.batch, self.dirs, self.g, tile=self.tile, waves=self.waves, out=self.grad,
                               ws=self.ws)

    def capture(self):
        s = torch.cuda.Stream(device=self.batch.device)
        s.wait_stream(torch.cuda.current_stream(self.batch.device))
        with torch.cuda.stream(s):
            self._enqueue()  # warm-up outside the graph
        torch.cuda.current_stream(self.batch.device).wait_stream(s)
        torch.cuda.synchronize(self.batch.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._enqueue()
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()
        return self.area, self.grad

    def status(self) -> int:
        return device_status(self.ws)
