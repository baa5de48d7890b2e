"""GPU test of d8_accum_noalloc (the entry point for callers that cannot
allocate): through the C ABI it must give the same results as d8_accum with a
caller workspace, on two calls in a row, the second with a smaller input (the
static scratch keeps the first call's contents)."""
import numpy as np
import pytest

import demgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

import paper_1605_05773_amd as d8  # noqa: E402
from gpu_util import assert_rel, dev, to_dev, to_np  # noqa: E402


@pytest.mark.parametrize("tile", [0, 32])
def test_noalloc_matches_accum_two_calls(tile):
    status = torch.full((1,), -1, dtype=torch.int32, device=dev())
    for H, W, seed in [(1500, 1700, 11), (700, 513, 12)]:
        print(f"[noalloc] tile {tile} shape {H}x{W} seed {seed}", flush=True)
        z = demgen.fbm_dem(H, W, sigma=8.0, seed=seed, nodata_frac=0.02, nodata_seed=seed)
        dirs = d8.flowdirs(to_dev(z))
        ref = d8.accum(dirs, tile=tile)
        out = torch.full((H, W), 0xDEAD, dtype=torch.uint32, device=dev())
        d8.accum_noalloc(dirs, out=out, tile=tile, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert np.array_equal(to_np(out), to_np(ref))
        w = to_dev(demgen.lognormal_f32((H, W), seed))
        refw = d8.accum(dirs, w, tile=tile)
        outw = torch.full((H, W), -1.0, dtype=torch.float32, device=dev())
        status.fill_(-1)
        d8.accum_noalloc(dirs, w, out=outw, tile=tile, status=status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        assert_rel(to_np(outw), to_np(refw), 1e-6, "noalloc weighted")


def test_noalloc_reports_data_errors():
    # a two-cell cycle: status bit 1 (cycle) comes back in the status word
    d = np.full((40, 50), 8, dtype=np.uint8)
    d[1:-1, 1:-1] = 2
    d[10, 10] = 0   # (10,10) -> E (10,11)
    d[10, 11] = 4   # (10,11) -> W (10,10)
    status = torch.zeros((1,), dtype=torch.int32, device=dev())
    out = torch.empty((40, 50), dtype=torch.uint32, device=dev())
    d8.accum_noalloc(to_dev(d), out=out, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & 2


def test_noalloc_refuses_shapes_beyond_scratch():
    big = torch.zeros((8192, 8192), dtype=torch.uint8, device=dev())
    out = torch.empty((8192, 8192), dtype=torch.uint32, device=dev())
    with pytest.raises(d8.D8Error) as e:
        d8.accum_noalloc(big, out=out)
    assert e.value.status == d8.D8_ENOMEM
