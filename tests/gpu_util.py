"""Helpers for the GPU parity tests (device transfers, comparisons)."""
import numpy as np
import torch

import paper_1605_05773_amd as d8


def dev():
    return torch.device("cuda", 0)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev())


def to_np(t):
    torch.cuda.synchronize()
    if t.dtype == torch.uint32:
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    return t.cpu().numpy()


def gpu_flowdirs(z):
    return to_np(d8.flowdirs(to_dev(z.astype(np.float32))))


def gpu_counts(dirs, tile=0):
    out = d8.accum(to_dev(dirs), tile=tile)
    res = to_np(out)
    assert d8.device_status() == d8.D8_OK
    return res


def gpu_weighted(dirs, w=None, tile=0, with_lo=False):
    wd = None if w is None else to_dev(w.astype(np.float32))
    H, W = dirs.shape
    out = torch.empty((H, W), dtype=torch.float32, device=dev())
    lo = torch.empty((H, W), dtype=torch.float32, device=dev()) if with_lo else None
    d8.accum(to_dev(dirs), wd, tile=tile, out=out, out_lo=lo)
    res = to_np(out)
    assert d8.device_status() == d8.D8_OK
    if with_lo:
        return res, to_np(lo)
    return res


def gpu_backward(dirs, g, tile=0):
    out = d8.accum_backward(to_dev(dirs), to_dev(g.astype(np.float32)), tile=tile)
    res = to_np(out)
    assert d8.device_status() == d8.D8_OK
    return res


def assert_rel(x, ref, rtol=1e-6, what=""):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(x - ref)
    bound = rtol * np.abs(ref)
    bad = err > bound
    if bad.any():
        i = np.argmax(err / np.maximum(np.abs(ref), 1e-300))
        raise AssertionError(f"{what}: {bad.sum()} cells exceed rel {rtol}; worst at {np.unravel_index(i, ref.shape)}"
                             f" got {x.flat[i]!r} ref {ref.flat[i]!r}")
