"""Seeded synthetic inputs for the D8 up-slope area workloads.

This module generates inputs only.  It holds none of the method's arithmetic
(no flow directions, no accumulation); both the oracle and the GPU path consume
what it returns.  Every array is a deterministic function of its parameters
and seed on a given machine (numpy PCG64 streams, scipy FFT).

Recipe (the paper publishes no dataset, so these stand in for real DEMs):

* fBm surface by spectral synthesis: complex Gaussian coefficients on the rfft
  half-plane with amplitude |k|^-(hurst+1) (k in cycles/cell, DC = 0,
  periodic), inverse FFT in float64, shifted to mean 0 and scaled to sample
  standard deviation sigma.
* plus a tilt 0.01*(x + y) in float64 (x = column, y = row), cast to float32.
* optional NoData (NaN) disks: centres uniform over the grid, integer radius
  uniform in [8, 64], added until at least the requested fraction is NaN.
* epsilon priority-flood fill (fill.c) in float32 with eps = 1e-3, which makes
  every interior cell strictly higher than one of its neighbours, i.e. the DEM
  has no pits and no flats (the paper's precondition, Sec. 3).
* the walled serpentine: one boustrophedon channel separated by walls, the
  adversarial case for dependency depth.
"""
from __future__ import annotations

import ctypes
import hashlib
import json
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_FILL_SO = os.path.join(_HERE, "_fill.so")
_fill_lib = None


def build_fill(force: bool = False) -> str:
    """Compile fill.c into _fill.so with gcc (host code, no GPU)."""
    src = os.path.join(_HERE, "fill.c")
    if force or not os.path.exists(_FILL_SO) or os.path.getmtime(_FILL_SO) < os.path.getmtime(src):
        tmp = _FILL_SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
        os.replace(tmp, _FILL_SO)
    return _FILL_SO


def _lib():
    global _fill_lib
    if _fill_lib is None:
        if not os.path.exists(_FILL_SO):
            raise RuntimeError("demgen/_fill.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_FILL_SO)
        lib.demgen_fill_eps.restype = ctypes.c_int
        lib.demgen_fill_eps.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_float,
                                        ctypes.c_int64]
        _fill_lib = lib
    return _fill_lib


def fill_eps(z: np.ndarray, eps: float = 1e-3) -> np.ndarray:
    """Epsilon priority-flood fill, in place on a C-contiguous float32 array."""
    assert z.dtype == np.float32 and z.flags.c_contiguous and z.ndim == 2
    n = z.shape[0] * z.shape[1]
    progress = (1 << 27) if n >= (1 << 28) else 0
    rc = _lib().demgen_fill_eps(z.ctypes.data, z.shape[0], z.shape[1], ctypes.c_float(eps), progress)
    if rc != 0:
        raise MemoryError("fill: allocation failed")
    return z


def fbm(rows: int, cols: int, hurst: float, sigma: float, seed: int) -> np.ndarray:
    """Spectral fBm in float64, mean 0, sample std sigma."""
    import scipy.fft

    rng = np.random.Generator(np.random.PCG64(seed))
    kc = cols // 2 + 1
    coef = np.empty((rows, kc), dtype=np.complex128)
    kx2 = np.fft.rfftfreq(cols) ** 2
    ky = np.fft.fftfreq(rows)
    block = 1024
    for r0 in range(0, rows, block):
        r1 = min(rows, r0 + block)
        k = np.sqrt(ky[r0:r1, None] ** 2 + kx2[None, :])
        with np.errstate(divide="ignore"):
            amp = np.where(k > 0, k ** (-(hurst + 1.0)), 0.0)
        re = rng.standard_normal((r1 - r0, kc))
        im = rng.standard_normal((r1 - r0, kc))
        coef[r0:r1].real = re * amp
        coef[r0:r1].imag = im * amp
        del k, amp, re, im
    z = scipy.fft.irfft2(coef, s=(rows, cols), workers=max(1, min(16, os.cpu_count() or 1)), overwrite_x=True)
    del coef
    z -= z.mean()
    sd = z.std()
    if sd > 0:
        z *= sigma / sd
    return z


def add_tilt_f32(z64: np.ndarray, slope: float = 0.01) -> np.ndarray:
    rows, cols = z64.shape
    out = np.empty((rows, cols), dtype=np.float32)
    x = np.arange(cols, dtype=np.float64)
    block = 1024
    for r0 in range(0, rows, block):
        r1 = min(rows, r0 + block)
        y = np.arange(r0, r1, dtype=np.float64)[:, None]
        out[r0:r1] = (z64[r0:r1] + slope * (x[None, :] + y)).astype(np.float32)
    return out


def nodata_disks(z: np.ndarray, frac: float, seed: int, rmin: int = 8, rmax: int = 64) -> int:
    """Set NaN disks in place until >= frac of the cells are NaN; returns disk count."""
    rows, cols = z.shape
    rng = np.random.Generator(np.random.PCG64(seed))
    target = int(math.ceil(frac * rows * cols))
    nan = int(np.isnan(z).sum())
    disks = 0
    while nan < target:
        r0 = int(rng.integers(0, rows))
        c0 = int(rng.integers(0, cols))
        rho = int(rng.integers(rmin, rmax + 1))
        ra, rb = max(0, r0 - rho), min(rows, r0 + rho + 1)
        ca, cb = max(0, c0 - rho), min(cols, c0 + rho + 1)
        rr = np.arange(ra, rb)[:, None] - r0
        cc = np.arange(ca, cb)[None, :] - c0
        m = rr * rr + cc * cc <= rho * rho
        sub = z[ra:rb, ca:cb]
        nan += int((m & ~np.isnan(sub)).sum())
        sub[m] = np.nan
        disks += 1
    return disks


def _say(msg):
    import sys

    print(f"[demgen] {msg}", file=sys.stderr, flush=True)


def fbm_dem(rows: int, cols: int, sigma: float, seed: int, hurst: float = 0.7, slope: float = 0.01,
            eps: float = 1e-3, nodata_frac: float = 0.0, nodata_seed: int = 0, fill: bool = True) -> np.ndarray:
    """The full DEM recipe: fBm + tilt -> float32 -> NoData disks -> eps fill
    (fill=False stops before the fill: the raw surface, with its pits and
    closed depressions, that conditioning starts from)."""
    big = rows * cols >= (1 << 26)
    z64 = fbm(rows, cols, hurst, sigma, seed)
    if big:
        _say(f"fbm {rows}x{cols} done")
    z = add_tilt_f32(z64, slope)
    del z64
    if nodata_frac > 0:
        nodata_disks(z, nodata_frac, nodata_seed)
    if fill:
        fill_eps(z, eps)
    return z


def serpentine(rows: int, cols: int) -> np.ndarray:
    """Walled serpentine DEM (float32).

    Channel rows are the odd rows 1, 3, ... <= rows-2, each over columns
    1..cols-2, alternately west->east and east->west.  The even rows between
    them are walls with a single gap cell at the end where the channel turns.
    Path cell k (k = 0 at the start) has the float32 whose bit pattern is
    0x3F800000 + (L-1-k), strictly decreasing to 1.0 at the last cell.  Walls
    and DEM-edge cells are 1e9; the edge cell beside the last path cell is 0.0
    (the single outlet that drains the whole interior).
    """
    assert rows >= 4 and cols >= 4
    z = np.full((rows, cols), 1e9, dtype=np.float32)
    ch = list(range(1, rows - 1, 2))
    path = []
    for i, r in enumerate(ch):
        cs = range(1, cols - 1) if i % 2 == 0 else range(cols - 2, 0, -1)
        path.extend((r, c) for c in cs)
        if i + 1 < len(ch):
            gap_c = cols - 2 if i % 2 == 0 else 1
            path.append((r + 1, gap_c))
    L = len(path)
    bits = (np.uint32(0x3F800000) + (np.uint32(L - 1) - np.arange(L, dtype=np.uint32))).astype(np.uint32)
    vals = bits.view(np.float32)
    pr = np.fromiter((p[0] for p in path), dtype=np.int64, count=L)
    pc = np.fromiter((p[1] for p in path), dtype=np.int64, count=L)
    z[pr, pc] = vals
    lr, lc = path[-1]
    out_c = cols - 1 if lc == cols - 2 else 0
    z[lr, out_c] = 0.0
    return z


def serpentine_fast(rows: int, cols: int) -> np.ndarray:
    """Same DEM as serpentine(), built with vectorised row writes (large sizes)."""
    assert rows >= 4 and cols >= 4
    z = np.full((rows, cols), 1e9, dtype=np.float32)
    ch = np.arange(1, rows - 1, 2)
    n = len(ch)
    seg = cols - 2
    L = n * seg + (n - 1)
    zbits = z.view(np.uint32)
    base = np.uint32(0x3F800000)
    k0 = 0
    cols_we = np.arange(1, cols - 1)
    for i, r in enumerate(ch):
        ks = k0 + np.arange(seg, dtype=np.int64)
        b = (base + (np.uint32(L - 1) - ks.astype(np.uint32))).astype(np.uint32)
        if i % 2 == 0:
            zbits[r, cols_we] = b
        else:
            zbits[r, cols_we[::-1]] = b
        k0 += seg
        if i + 1 < n:
            gap_c = cols - 2 if i % 2 == 0 else 1
            zbits[r + 1, gap_c] = base + np.uint32(L - 1 - k0)
            k0 += 1
    last_r = ch[-1]
    last_c = cols - 2 if (n - 1) % 2 == 0 else 1
    out_c = cols - 1 if last_c == cols - 2 else 0
    z[last_r, out_c] = 0.0
    return z


def lognormal_f32(shape, seed: int, mu: float = 0.0, s: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.lognormal(mu, s, size=shape).astype(np.float32)


def normal_f64(shape, seed: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=shape)


def batch_shapes(n: int, seed: int, lo: int = 64, hi: int = 2048):
    """Sides log-uniform in [lo, hi] with aspect ratio uniform in 1:1..1:4."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        long_side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        a = rng.uniform(1.0, 4.0)
        short = max(16, int(round(long_side / a)))
        if rng.integers(0, 2):
            out.append((long_side, short))
        else:
            out.append((short, long_side))
    return out


# ---------------------------------------------------------------- workloads --

CONFIGS = {
    # name: (rows, cols, kwargs for fbm_dem)
    "c0": (512, 512, dict(sigma=5.0, seed=0)),
    "c1": (8192, 8192, dict(sigma=20.0, seed=1, nodata_frac=0.05, nodata_seed=101)),
    "c2a": (32768, 32768, dict(sigma=50.0, seed=2)),
    "c3": (4096, 4096, dict(sigma=5.0, seed=3)),
}


def _cache_dir():
    d = os.environ.get("D8_CACHE", "/tmp/d8_dem_cache")
    os.makedirs(d, exist_ok=True)
    return d


def cached(name: str, params: dict, make):
    """Memoise a generated float32/uint8 array on local disk (raw + sha256 + params)."""
    key = hashlib.sha256(json.dumps([name, params], sort_keys=True).encode()).hexdigest()[:16]
    d = _cache_dir()
    path = os.path.join(d, f"{name}_{key}.npy")
    meta = path + ".json"
    if os.path.exists(path) and os.path.exists(meta):
        with open(meta) as f:
            m = json.load(f)
        arr = np.load(path, mmap_mode="r")
        return np.ascontiguousarray(arr), m
    arr = make()
    tmp = path + ".tmp%d.npy" % os.getpid()
    np.save(tmp, arr)
    os.replace(tmp, path)
    h = hashlib.sha256(memoryview(np.ascontiguousarray(arr)).cast("B")).hexdigest()
    m = {"name": name, "params": params, "shape": list(arr.shape), "dtype": str(arr.dtype), "sha256": h}
    with open(meta, "w") as f:
        json.dump(m, f)
    return arr, m


def config_dem(name: str, use_cache: bool = True, raw: bool = False) -> np.ndarray:
    """DEM for a named workload (c0, c1, c2a, c3, c2b = serpentine 16384^2).
    raw=True: the same surface before the epsilon fill (fBm workloads only)."""
    if raw:
        rows, cols, kw = CONFIGS[name]
        params = dict(rows=rows, cols=cols, raw=True, **kw)
        mk = lambda: fbm_dem(rows, cols, fill=False, **kw)
    elif name == "c2b":
        params = {"rows": 16384, "cols": 16384}
        mk = lambda: serpentine_fast(16384, 16384)
    else:
        rows, cols, kw = CONFIGS[name]
        params = dict(rows=rows, cols=cols, **kw)
        mk = lambda: fbm_dem(rows, cols, **kw)
    if not use_cache:
        return mk()
    arr, _ = cached(name, params, mk)
    return arr


def c4_batch(n: int = 512, sizes_seed: int = 4):
    """The batched workload: n DEMs of uneven shape, each from the 512^2 recipe."""
    shapes = batch_shapes(n, sizes_seed)
    dems = [fbm_dem(r, c, sigma=5.0, seed=10000 + i) for i, (r, c) in enumerate(shapes)]
    w = [lognormal_f32((r, c), 20000 + i) for i, (r, c) in enumerate(shapes)]
    g = [lognormal_f32((r, c), 30000 + i) for i, (r, c) in enumerate(shapes)]
    return shapes, dems, w, g
