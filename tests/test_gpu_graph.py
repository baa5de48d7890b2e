"""Batched launch captured as a HIP graph, and the autotuner (with its cache).

Replays are checked against the oracle and against eager calls, with eager
work and synchronisations between replays, and with inputs rewritten in
place between replays."""
import json

import numpy as np
import pytest

import demgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

import paper_1605_05773_amd as d8  # noqa: E402
from gpu_util import assert_rel, dev, to_dev, to_np  # noqa: E402


@pytest.fixture(scope="module")
def small_batch():
    shapes = demgen.batch_shapes(24, 41, lo=16, hi=300)
    dems = [demgen.fbm_dem(r, c, sigma=5.0, seed=700 + i) for i, (r, c) in enumerate(shapes)]
    dirs = [oracle.flowdirs(z) for z in dems]
    return shapes, dirs


def test_graph_replays_match_oracle_and_eager(small_batch):
    shapes, dirs = small_batch
    b = d8.Batch(shapes, dev())
    gr = d8.BatchedGraph(b)
    gr.dirs.copy_(b.pack([to_dev(x) for x in dirs], torch.uint8))
    for rep in range(3):
        ws = [demgen.lognormal_f32(s, 900 + 10 * rep + i) for i, s in enumerate(shapes)]
        gs = [demgen.lognormal_f32(s, 950 + 10 * rep + i) for i, s in enumerate(shapes)]
        gr.w.copy_(b.pack([to_dev(x) for x in ws], torch.float32))
        gr.g.copy_(b.pack([to_dev(x) for x in gs], torch.float32))
        area, grad = gr.replay()
        torch.cuda.synchronize()
        assert gr.status() == d8.D8_OK
        # eager calls on the same inputs, between replays
        ea = d8.accum_batched(b, gr.dirs, gr.w)
        eg = d8.accum_backward_batched(b, gr.dirs, gr.g)
        torch.cuda.synchronize()
        for i in range(len(shapes)):
            A = to_np(b.unpack(area)[i])
            G = to_np(b.unpack(grad)[i])
            assert_rel(A, oracle.accum_f64(dirs[i], ws[i]), 1e-6, f"replay {rep} area {i}")
            assert_rel(G, oracle.backward_f64(dirs[i], gs[i]), 1e-6, f"replay {rep} grad {i}")
            assert_rel(A, to_np(b.unpack(ea)[i]), 1e-6, f"replay {rep} vs eager area {i}")
            assert_rel(G, to_np(b.unpack(eg)[i]), 1e-6, f"replay {rep} vs eager grad {i}")


def test_autotune_and_cache(small_batch, tmp_path):
    shapes, dirs = small_batch
    b = d8.Batch(shapes, dev())
    dp = b.pack([to_dev(x) for x in dirs], torch.uint8)
    wp = b.pack([to_dev(demgen.lognormal_f32(s, 10 + i)) for i, s in enumerate(shapes)], torch.float32)
    cache = tmp_path / "tune.json"
    t, w, ms = d8.autotune_batched(b, dp, wp, cache_path=str(cache))
    assert (t == 32 and w in (1, 2, 4)) or (t == 64 and w in (2, 4, 8, 16))
    assert ms > 0
    stored = json.loads(cache.read_text())
    assert list(stored.values()) == [{"tile": t, "waves": w, "ms": ms}]
    assert d8.autotune_batched(b, dp, wp, cache_path=str(cache)) == (t, w, ms)
    # the tuned configuration gives the oracle's results
    A = b.unpack(d8.accum_batched(b, dp, wp, tile=t, waves=w))
    for i in range(len(shapes)):
        w_i = to_np(b.unpack(wp)[i])
        assert_rel(to_np(A[i]), oracle.accum_f64(dirs[i], w_i), 1e-6, f"tuned {i}")
