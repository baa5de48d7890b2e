"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point the header declares, and rejects bad arguments before any
device work."""
import ctypes
import os
import re

import pytest

import paper_1605_05773_amd as d8

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "d8.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(d8_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(d8.LIB_PATH):
        pytest.skip("libd8.so not built")
    L = d8.lib()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(d8.EXPORTED)


def test_version_and_strerror():
    L = d8.lib()
    assert L.d8_version().startswith(b"d8-gfx950")
    for s in range(7):
        assert len(L.d8_strerror(s)) > 1


def test_workspace_bytes_validation():
    L = d8.lib()
    assert L.d8_workspace_bytes(0, 10, 0) == 0
    assert L.d8_workspace_bytes(10, -1, 0) == 0
    assert L.d8_workspace_bytes(10, 10, 48) == 0
    assert L.d8_workspace_bytes(1 << 17, 1 << 16, 0) == 0          # > 2^32 - 1 cells
    assert L.d8_workspace_bytes(1, 1 << 31, 0) == 0                # a side > 2^31 - 1
    assert L.d8_workspace_bytes(65535, 65537, 0) > 0               # 2^32 - 1 cells
    a = L.d8_workspace_bytes(1000, 1000, 64)
    b = L.d8_workspace_bytes(1000, 1000, 32)
    assert 0 < a < b                                               # smaller tiles, more perimeter slots
    assert L.d8_workspace_bytes(1, 1, 32) > 0
    # the backward: the forward's workspace plus 6 bytes per cell
    assert L.d8_backward_workspace_bytes(1000, 1000, 64) >= L.d8_workspace_bytes(1000, 1000, 64) + 6 * 1000 * 1000
    assert L.d8_backward_workspace_bytes(0, 10, 0) == 0
    assert L.d8_backward_workspace_bytes(10, 10, 48) == 0


def test_argument_errors_before_device_work():
    L = d8.lib()
    fake = ctypes.c_void_p(0x1000)
    assert L.d8_accum(None, 10, 10, None, d8.D8_U32, fake, None, fake, 1 << 30, 0, None) == d8.D8_EINVAL
    assert L.d8_accum(fake, 10, 10, None, 7, fake, None, fake, 1 << 30, 0, None) == d8.D8_EINVAL
    assert L.d8_accum(fake, 10, 10, fake, d8.D8_U32, fake, None, fake, 1 << 30, 0, None) == d8.D8_EINVAL
    assert L.d8_accum(fake, 0, 10, None, d8.D8_U32, fake, None, fake, 1 << 30, 0, None) == d8.D8_EINVAL
    # workspace pointer not 256-byte aligned
    assert L.d8_accum(fake, 10, 10, None, d8.D8_U32, fake, None, ctypes.c_void_p(0x1010), 1 << 30, 0,
                      None) == d8.D8_EINVAL
    # workspace too small
    assert L.d8_accum(fake, 100, 100, None, d8.D8_U32, fake, None, fake, 16, 0, None) == d8.D8_ENOMEM
    # weighted with a 128 tile is not provided
    assert L.d8_accum(fake, 100, 100, None, d8.D8_F32, fake, None, fake, 1 << 30, 128, None) == d8.D8_EUNSUPPORTED
    assert L.d8_accum_backward(fake, 10, 10, None, fake, fake, 1 << 30, 0, None) == d8.D8_EINVAL
    assert L.d8_flowdirs(None, 10, 10, fake, None) == d8.D8_EINVAL
    assert L.d8_flowdirs(fake, 1 << 20, 1 << 13, fake, None) == d8.D8_EINVAL
    assert L.d8_flowdirs_steepest(None, 10, 10, fake, None) == d8.D8_EINVAL
    assert L.d8_accum_dem(None, 10, 10, fake, fake, fake, 1 << 20, 0, None) == d8.D8_EINVAL
    assert L.d8_accum_dem(fake, 10, 10, None, fake, fake, 1 << 20, 0, None) == d8.D8_EINVAL
    assert L.d8_flowdirs_steepest(fake, 0, 10, fake, None) == d8.D8_EINVAL
    assert L.d8_device_status(None, None, None) == d8.D8_EINVAL
    # the no-allocation variant: same argument rules, and shapes beyond its
    # static scratch are refused before any device work
    assert L.d8_accum_noalloc(None, 10, 10, None, d8.D8_U32, fake, None, 0, None, None) == d8.D8_EINVAL
    assert L.d8_accum_noalloc(fake, 10, 10, fake, d8.D8_U32, fake, None, 0, None, None) == d8.D8_EINVAL
    assert L.d8_accum_noalloc(fake, 0, 10, None, d8.D8_U32, fake, None, 0, None, None) == d8.D8_EINVAL
    assert L.d8_accum_noalloc(fake, 8192, 8192, None, d8.D8_U32, fake, None, 0, None, None) == d8.D8_ENOMEM
    assert L.d8_workspace_bytes(5900, 5900, 64) <= 64 << 20 < L.d8_workspace_bytes(8192, 8192, 64)


def test_batched_workspace_validation():
    L = d8.lib()
    descs = (d8.d8_desc * 2)(d8.d8_desc(0, 10, 20), d8.d8_desc(200, 30, 5))
    assert L.d8_batched_workspace_bytes(ctypes.addressof(descs), 2, 64) > 0
    # backward: 6 bytes per packed cell up to the largest offset + rows * cols (200 + 150)
    assert (L.d8_batched_backward_workspace_bytes(ctypes.addressof(descs), 2, 64)
            >= L.d8_batched_workspace_bytes(ctypes.addressof(descs), 2, 64) + 6 * 350)
    bad = (d8.d8_desc * 1)(d8.d8_desc(0, 0, 20))
    assert L.d8_batched_workspace_bytes(ctypes.addressof(bad), 1, 64) == 0
    assert L.d8_batched_workspace_bytes(ctypes.addressof(descs), 0, 64) == 0


def test_fill_argument_errors_before_device_work():
    L = d8.lib()
    fake = ctypes.c_void_p(0x10000)
    out = ctypes.c_void_p(0x900000)
    ws = ctypes.c_void_p(0x1000000)
    assert L.d8_fill_workspace_bytes(0, 5) == 0
    assert L.d8_fill_workspace_bytes(1 << 17, 1 << 16) == 0
    nb = L.d8_fill_workspace_bytes(100, 100)
    assert nb >= 256 + 3 * 4 * 4 and nb % 256 == 0
    assert L.d8_fill_workspace_bytes(1000, 1000) > nb
    f = L.d8_fill_eps
    c = ctypes.c_float
    assert f(None, 100, 100, c(1e-3), out, ws, nb, None, None) == d8.D8_EINVAL
    assert f(fake, 100, 100, c(1e-3), None, ws, nb, None, None) == d8.D8_EINVAL
    assert f(fake, 0, 100, c(1e-3), out, ws, nb, None, None) == d8.D8_EINVAL
    for bad in (0.0, -1e-3, float("nan"), float("inf"), 1e-40):     # eps must be a positive normal float
        assert f(fake, 100, 100, c(bad), out, ws, nb, None, None) == d8.D8_EINVAL, bad
    # out overlapping dem (same buffer, and a partial overlap)
    assert f(fake, 100, 100, c(1e-3), fake, ws, nb, None, None) == d8.D8_EINVAL
    assert f(fake, 100, 100, c(1e-3), ctypes.c_void_p(0x10000 + 400), ws, nb, None, None) == d8.D8_EINVAL
    assert f(fake, 100, 100, c(1e-3), out, ctypes.c_void_p(0x1000010), nb, None, None) == d8.D8_EINVAL
    assert f(fake, 100, 100, c(1e-3), out, ws, nb - 1, None, None) == d8.D8_ENOMEM


def test_streamed_argument_errors_before_device_work():
    L = d8.lib()
    assert L.d8_accum_streamed_workspace_bytes(100, 100, 0) == 0
    assert L.d8_accum_streamed_workspace_bytes(100, 100, 100) == 0      # not a multiple of 64
    assert L.d8_accum_streamed_workspace_bytes(0, 100, 64) == 0
    a = L.d8_accum_streamed_workspace_bytes(1000, 1000, 64)
    b = L.d8_accum_streamed_workspace_bytes(1000, 1000, 256)
    assert L.d8_workspace_bytes(1000, 1000, 64) < a < b
    # a strip taller than the DEM is clipped to it
    assert L.d8_accum_streamed_workspace_bytes(100, 100, 6400) == L.d8_accum_streamed_workspace_bytes(100, 100, 128)
    host = (ctypes.c_uint8 * 16)()
    out = (ctypes.c_uint32 * 16)()
    ws = ctypes.c_void_p(0x1000000)
    f = L.d8_accum_streamed
    assert f(None, 4, 4, out, 64, ws, 1 << 30, None) == d8.D8_EINVAL
    assert f(host, 4, 4, None, 64, ws, 1 << 30, None) == d8.D8_EINVAL
    assert f(host, 4, 4, out, 32, ws, 1 << 30, None) == d8.D8_EINVAL
    assert f(host, 4, 4, out, 64, ctypes.c_void_p(0x1000010), 1 << 30, None) == d8.D8_EINVAL
    assert f(host, 4, 4, out, 64, ws, 16, None) == d8.D8_ENOMEM


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
