"""CPU oracle for D8 flow directions and up-slope area -- TEST INFRASTRUCTURE.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  The product path never does; it shares no code with it.

Thin numpy wrappers over d8_oracle.c (plain single-threaded C, fp64 sums), plus
O(N) checkers of the recursion identity (Eq. 1) and the outlet-sum invariant.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")
_lib = None

OK, NOMEM, BADDIR, CYCLE = 0, 2, 4, 5

# Offsets (dr, dc) of direction codes 0..7: E, NE, N, NW, W, SW, S, SE (row 0 = north).
DR = np.array([0, -1, -1, -1, 0, 1, 1, 1], dtype=np.int64)
DC = np.array([1, 1, 0, -1, -1, -1, 0, 1], dtype=np.int64)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__({BADDIR: "bad direction field", CYCLE: "cycle", NOMEM: "out of memory"}.get(status, str(status)))
        self.status = status


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "d8_oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError("oracle/_oracle.so is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(_SO)
        P, I = ctypes.c_void_p, ctypes.c_int64
        for name in ("orc_flowdirs", "orc_flowdirs_steepest", "orc_accum_u32", "orc_accum_f64", "orc_backward_f64",
                     "orc_bruteforce_f64", "orc_backward_f64d", "orc_accum_f64d"):
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
        L.orc_flowdirs.argtypes = [P, I, I, P]
        L.orc_flowdirs_steepest.argtypes = [P, I, I, P]
        L.orc_accum_u32.argtypes = [P, I, I, P]
        L.orc_accum_f64.argtypes = [P, I, I, P, P]
        L.orc_accum_f64d.argtypes = [P, I, I, P, P]
        L.orc_backward_f64.argtypes = [P, I, I, P, P]
        L.orc_backward_f64d.argtypes = [P, I, I, P, P]
        L.orc_bruteforce_f64.argtypes = [P, I, I, P, P]
        L.orc_fill_eps.restype = ctypes.c_int
        L.orc_fill_eps.argtypes = [P, I, I, ctypes.c_float, P]
        L.orc_depth.restype = ctypes.c_int64
        L.orc_depth.argtypes = [P, I, I]
        _lib = L
    return _lib


def _c(a, dt):
    a = np.ascontiguousarray(a, dtype=dt)
    return a


def _ptr(a):
    return None if a is None else a.ctypes.data


def _check(st):
    if st != OK:
        raise OracleError(st)


def flowdirs(z: np.ndarray, rule: str = "lowest") -> np.ndarray:
    """D8 codes: rule "lowest" (lowest of eight) or "steepest" (largest drop
    over distance, diagonals at sqrt 2)."""
    z = _c(z, np.float32)
    out = np.empty(z.shape, dtype=np.uint8)
    fn = {"lowest": lib().orc_flowdirs, "steepest": lib().orc_flowdirs_steepest}[rule]
    _check(fn(z.ctypes.data, z.shape[0], z.shape[1], out.ctypes.data))
    return out


def fill_eps(z: np.ndarray, eps: float = 1e-3) -> np.ndarray:
    """Epsilon-filled DEM (float32): the unique F with F = z on seeds (valid
    cells on the DEM boundary or next to NaN) and F(c) = max(z(c), min over
    valid neighbours of inc(F(n))) elsewhere, inc(x) = fl32(x + eps) or the
    next float above x.  Dijkstra order in d8_oracle.c.  NaN stays NaN."""
    z = _c(z, np.float32)
    out = np.empty(z.shape, dtype=np.float32)
    _check(lib().orc_fill_eps(z.ctypes.data, z.shape[0], z.shape[1], ctypes.c_float(eps), out.ctypes.data))
    return out


def accum_u32(dirs: np.ndarray) -> np.ndarray:
    d = _c(dirs, np.uint8)
    out = np.empty(d.shape, dtype=np.uint32)
    _check(lib().orc_accum_u32(d.ctypes.data, d.shape[0], d.shape[1], out.ctypes.data))
    return out


def accum_f64(dirs: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    d = _c(dirs, np.uint8)
    out = np.empty(d.shape, dtype=np.float64)
    if w is not None and np.asarray(w).dtype == np.float64:
        wd = _c(w, np.float64)
        _check(lib().orc_accum_f64d(d.ctypes.data, d.shape[0], d.shape[1], wd.ctypes.data, out.ctypes.data))
        return out
    wf = None if w is None else _c(w, np.float32)
    _check(lib().orc_accum_f64(d.ctypes.data, d.shape[0], d.shape[1], _ptr(wf), out.ctypes.data))
    return out


def backward_f64(dirs: np.ndarray, g: np.ndarray | None = None) -> np.ndarray:
    d = _c(dirs, np.uint8)
    out = np.empty(d.shape, dtype=np.float64)
    if g is not None and np.asarray(g).dtype == np.float64:
        gd = _c(g, np.float64)
        _check(lib().orc_backward_f64d(d.ctypes.data, d.shape[0], d.shape[1], gd.ctypes.data, out.ctypes.data))
        return out
    gf = None if g is None else _c(g, np.float32)
    _check(lib().orc_backward_f64(d.ctypes.data, d.shape[0], d.shape[1], _ptr(gf), out.ctypes.data))
    return out


def bruteforce_f64(dirs: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    d = _c(dirs, np.uint8)
    wf = None if w is None else _c(w, np.float32)
    out = np.empty(d.shape, dtype=np.float64)
    _check(lib().orc_bruteforce_f64(d.ctypes.data, d.shape[0], d.shape[1], _ptr(wf), out.ctypes.data))
    return out


def depth(dirs: np.ndarray) -> int:
    d = _c(dirs, np.uint8)
    r = lib().orc_depth(d.ctypes.data, d.shape[0], d.shape[1])
    if r < 0:
        raise OracleError(CYCLE)
    return int(r)


# ------------------------------------------------------------ O(N) checkers --

def targets(dirs: np.ndarray) -> np.ndarray:
    """Flat target index per cell (-1 for outlets / NoData).  Assumes a valid field."""
    H, W = dirs.shape
    d = dirs.reshape(-1).astype(np.int64)
    idx = np.arange(H * W, dtype=np.int64)
    r, c = idx // W, idx % W
    live = d < 8
    k = np.where(live, d, 0)
    t = (r + DR[k]) * W + (c + DC[k])
    return np.where(live, t, -1)


def identity_residual(dirs: np.ndarray, A: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """Eq. (1) residual per cell: A(p) - w(p) - sum of A over the cells draining into p.
    Computed in fp64 (counts are exact below 2^53)."""
    H, W = dirs.shape
    t = targets(dirs)
    a = A.reshape(-1).astype(np.float64)
    src = t >= 0
    inflow = np.bincount(t[src], weights=a[src], minlength=H * W)
    valid = dirs.reshape(-1) != 255
    ww = np.where(valid, 1.0 if w is None else np.asarray(w, dtype=np.float64).reshape(-1), 0.0)
    return (a - ww - inflow).reshape(H, W)


def outlet_total(dirs: np.ndarray, A: np.ndarray) -> float:
    """Sum of A over outlet cells (code 8); equals the total weight for a valid field."""
    m = dirs == 8
    return float(A[m].astype(np.float64).sum())
