"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Counts and flow directions must match bit for bit; weighted results and
gradients within 1e-6 relative of fp64 (the tolerance the method's weighted
form is held to; the tile passes and the resolve sum in fp64 and round once to
float32, so the observed error is far below it).
"""
import numpy as np
import pytest

import demgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

import paper_1605_05773_amd as d8  # noqa: E402
from golden_io import load  # noqa: E402
from gpu_util import (assert_rel, dev, gpu_backward, gpu_counts, gpu_flowdirs, gpu_weighted, to_dev,  # noqa: E402
                      to_np)

TILES = [32, 64, 128]


def random_dem(H, W, seed, nan_frac=0.0):
    rng = np.random.default_rng(seed)
    z = rng.random((H, W)).astype(np.float32)
    if nan_frac:
        z[rng.random((H, W)) < nan_frac] = np.nan
    return z


# ------------------------------------------------------------------ flowdirs

@pytest.mark.parametrize("name", ["hand_4x5.txt", "hand_5x5_nodata_tie.txt"])
def test_golden_fixtures(name):
    dem, dirs_exp, area_exp = load(name)
    d = gpu_flowdirs(dem)
    np.testing.assert_array_equal(d, dirs_exp)
    for t in TILES:
        np.testing.assert_array_equal(gpu_counts(d, t), area_exp)


@pytest.mark.parametrize("shape,nan", [((1, 1), 0), ((1, 37), 0), ((37, 1), 0), ((3, 3), 0), ((70, 131), 0),
                                       ((129, 67), 0.2), ((256, 300), 0.05)])
@pytest.mark.parametrize("seed", [0, 1])
def test_flowdirs_random(shape, nan, seed):
    z = random_dem(*shape, seed, nan)
    np.testing.assert_array_equal(gpu_flowdirs(z), oracle.flowdirs(z))


def test_flowdirs_c0_and_ties():
    z = demgen.config_dem("c0")
    np.testing.assert_array_equal(gpu_flowdirs(z), oracle.flowdirs(z))
    y, x = np.mgrid[0:33, 0:45].astype(np.float32)
    for a, b in [(0.01, 0.0), (0.0, 0.01), (-0.01, 0.0), (0.0, -0.01)]:
        zp = (np.float32(a) * x + np.float32(b) * y).astype(np.float32)
        np.testing.assert_array_equal(gpu_flowdirs(zp), oracle.flowdirs(zp))


@pytest.mark.parametrize("shape,nan", [((1, 1), 0), ((3, 3), 0), ((70, 131), 0), ((129, 67), 0.2), ((300, 257), 0.02)])
@pytest.mark.parametrize("seed", [0, 3])
def test_flowdirs_steepest_random(shape, nan, seed):
    z = random_dem(*shape, seed, nan)
    np.testing.assert_array_equal(to_np(d8.flowdirs(to_dev(z), rule="steepest")), oracle.flowdirs(z, rule="steepest"))


def test_flowdirs_steepest_planes_and_c0():
    y, x = np.mgrid[0:40, 0:37].astype(np.float64)
    for a, b in [(0.01, 0.004), (0.004, 0.01), (0.01, 0.0), (-0.01, 0.004), (0.003, -0.02)]:
        z = (a * x + b * y).astype(np.float32)
        np.testing.assert_array_equal(to_np(d8.flowdirs(to_dev(z), rule="steepest")),
                                      oracle.flowdirs(z, rule="steepest"))
    z = demgen.config_dem("c0")
    d = oracle.flowdirs(z, rule="steepest")
    dg = d8.flowdirs(to_dev(z), rule="steepest")
    np.testing.assert_array_equal(to_np(dg), d)
    assert (d != oracle.flowdirs(z)).any()  # the two rules differ on real terrain
    np.testing.assert_array_equal(to_np(d8.accum(dg)), oracle.accum_u32(d))


# ------------------------------------------------------------------- counts

@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("shape,nan", [((1, 1), 0), ((1, 300), 0), ((300, 1), 0), ((2, 2), 0), ((33, 33), 0),
                                       ((65, 63), 0.1), ((130, 257), 0), ((200, 129), 0.3)])
def test_counts_random(tile, shape, nan):
    z = random_dem(*shape, 7, nan)
    d = oracle.flowdirs(z)
    np.testing.assert_array_equal(gpu_counts(d, tile), oracle.accum_u32(d))


@pytest.mark.parametrize("tile", TILES)
def test_counts_c0_all_tiles(tile):
    d = oracle.flowdirs(demgen.config_dem("c0"))
    np.testing.assert_array_equal(gpu_counts(d, tile), oracle.accum_u32(d))


@pytest.mark.parametrize("shape", [(16, 16), (40, 33), (130, 130), (256, 256), (300, 97)])
@pytest.mark.parametrize("tile", TILES)
def test_counts_serpentine(shape, tile):
    d = oracle.flowdirs(demgen.serpentine(*shape))
    np.testing.assert_array_equal(gpu_counts(d, tile), oracle.accum_u32(d))


def test_counts_c0_like_nodata_and_ragged():
    z = demgen.fbm_dem(1000, 777, sigma=20.0, seed=5, nodata_frac=0.05, nodata_seed=6)
    d = oracle.flowdirs(z)
    ref = oracle.accum_u32(d)
    for t in TILES:
        np.testing.assert_array_equal(gpu_counts(d, t), ref)


@pytest.mark.parametrize("shape", [(256, 320), (200, 260), (192, 258), (131, 516)])
def test_counts_fixup_grouped_and_single_paths(shape):
    """The finalising pass moves counts 4 cells at a time on whole 64x64
    tiles whose rows start on a 4-cell boundary and cell by cell elsewhere:
    all tiles grouped (256x320), grouped and ragged tiles mixed (200x260,
    131x516), no row aligned (192x258).  Both give the oracle's counts."""
    z = demgen.fbm_dem(*shape, sigma=5.0, seed=sum(shape), nodata_frac=0.02, nodata_seed=3)
    d = oracle.flowdirs(z)
    np.testing.assert_array_equal(gpu_counts(d, 64), oracle.accum_u32(d))


def converging_valleys(H, W, spacing=64, offset=27):
    """A direction field of parallel valleys: every cell drains south, towards
    the nearest valley column diagonally (SE or SW) and straight down it, so
    that the paths entering a tile through its top row run into the valley in
    lockstep (two receivers reach the same valley cell at the same step, in
    long runs) and the finalising walks merge lanes pair after pair."""
    d = np.full((H, W), 6, dtype=np.uint8)  # S
    c = np.arange(W)
    ch = offset + spacing * np.round((c - offset) / spacing).astype(np.int64)
    d[:, c < ch] = 7  # SE
    d[:, c > ch] = 5  # SW
    d[0, :] = d[-1, :] = 8
    d[:, 0] = d[:, -1] = 8
    return d


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("shape,spacing,offset", [((320, 300), 64, 27), ((257, 513), 40, 5), ((200, 130), 130, 64)])
def test_counts_converging_walks(tile, shape, spacing, offset):
    d = converging_valleys(*shape, spacing, offset)
    np.testing.assert_array_equal(gpu_counts(d, tile), oracle.accum_u32(d))


@pytest.mark.parametrize("tile", [32, 64])
def test_weighted_converging_walks(tile):
    d = converging_valleys(320, 300, 64, 27)
    w = np.random.default_rng(11).lognormal(0.0, 1.0, d.shape).astype(np.float32)
    assert_rel(gpu_weighted(d, w, tile), oracle.accum_f64(d, w), 1e-6)


def test_counts_deterministic_and_tile_invariant():
    d = oracle.flowdirs(demgen.fbm_dem(777, 1000, sigma=5.0, seed=9))
    runs = [gpu_counts(d, t) for t in (32, 64, 64, 128)]
    for r in runs[1:]:
        np.testing.assert_array_equal(r, runs[0])


@pytest.mark.parametrize("tile", TILES)
@pytest.mark.parametrize("shape,nan", [((1, 1), 0), ((2, 300), 0), ((65, 63), 0.1), ((130, 257), 0), ((200, 129), 0.3),
                                       ((300, 301), 0.02)])
def test_accum_dem_fused(tile, shape, nan):
    z = random_dem(*shape, 11, nan)
    d = oracle.flowdirs(z)
    counts, dirs = d8.accum_dem(to_dev(z), tile=tile)
    assert d8.device_status() == d8.D8_OK
    np.testing.assert_array_equal(to_np(dirs), d)
    np.testing.assert_array_equal(to_np(counts), oracle.accum_u32(d))


def test_accum_dem_fused_c0_nodata():
    z = demgen.fbm_dem(700, 650, sigma=20.0, seed=5, nodata_frac=0.05, nodata_seed=6)
    d = oracle.flowdirs(z)
    for t in TILES:
        counts, dirs = d8.accum_dem(to_dev(z), tile=t)
        np.testing.assert_array_equal(to_np(dirs), d)
        np.testing.assert_array_equal(to_np(counts), oracle.accum_u32(d))


# ----------------------------------------------------------------- weighted

@pytest.mark.parametrize("tile", [32, 64])
def test_weighted_c0(tile):
    d = oracle.flowdirs(demgen.config_dem("c0"))
    w = demgen.lognormal_f32(d.shape, 303)
    ref = oracle.accum_f64(d, w)
    out, lo = gpu_weighted(d, w, tile, with_lo=True)
    assert_rel(out, ref, 1e-6, "weighted")
    # the (out, out_lo) pair carries far more than float32 precision
    assert_rel(out.astype(np.float64) + lo.astype(np.float64), ref, 1e-10, "weighted hi+lo")


@pytest.mark.parametrize("tile", [32, 64])
def test_weighted_unit_equals_counts(tile):
    d = oracle.flowdirs(demgen.fbm_dem(300, 301, sigma=5.0, seed=2))
    counts = oracle.accum_u32(d)
    assert counts.max() < 2 ** 24
    out = gpu_weighted(d, None, tile)
    np.testing.assert_array_equal(out, counts.astype(np.float32))


@pytest.mark.parametrize("shape,nan", [((1, 1), 0), ((1, 90), 0), ((90, 1), 0), ((70, 131), 0.1)])
def test_weighted_random_shapes(shape, nan):
    z = random_dem(*shape, 3, nan)
    d = oracle.flowdirs(z)
    w = demgen.lognormal_f32(shape, 4)
    for t in (32, 64):
        assert_rel(gpu_weighted(d, w, t), oracle.accum_f64(d, w), 1e-6, "weighted")


def test_weighted_serpentine_deep():
    d = oracle.flowdirs(demgen.serpentine(256, 256))
    w = demgen.lognormal_f32(d.shape, 8)
    assert_rel(gpu_weighted(d, w, 32), oracle.accum_f64(d, w), 1e-6, "weighted serpentine")


def test_weighted_linearity():
    d = oracle.flowdirs(demgen.fbm_dem(200, 250, sigma=5.0, seed=1))
    w1 = demgen.lognormal_f32(d.shape, 1)
    w2 = demgen.lognormal_f32(d.shape, 2)
    a = gpu_weighted(d, w1).astype(np.float64) + gpu_weighted(d, w2).astype(np.float64)
    b = gpu_weighted(d, (w1 + w2).astype(np.float32)).astype(np.float64)
    ref = oracle.accum_f64(d, w1.astype(np.float64) + w2.astype(np.float64))
    assert_rel(a, ref, 2e-6, "linearity sum")
    assert_rel(b, oracle.accum_f64(d, (w1 + w2).astype(np.float32)), 1e-6, "linearity")


@pytest.mark.parametrize("tile", [32, 64])
def test_weighted_run_to_run_variation_bounded(tile):
    """Weighted sums are fp64 with atomic additions, so their order (and the
    last bits of the sum) can change from run to run.  Every order of adding
    n nonnegative terms is within (n-1)u of the exact sum (u = 2^-53), and a
    (out, out_lo) pair carries an fp64 value to 2^-48 relative (the tile-local
    value passes through one such pair before the inflow is added), so a run
    is within (n-1)u + 2^-47 of the exact sum and two runs, or a run and the
    fp64 oracle, differ by at most twice that, relative, at a cell with n
    upstream cells; float32 `out` itself may differ by one ulp only where the
    fp64 sum sits that close to a float32 rounding boundary."""
    d = oracle.flowdirs(demgen.fbm_dem(1024, 1000, sigma=8.0, seed=5))
    w = demgen.lognormal_f32(d.shape, 17)
    n = oracle.accum_u32(d).astype(np.float64)
    ref = oracle.accum_f64(d, w)
    bound = 2.0 * (np.maximum(n - 1.0, 0.0) * 2.0 ** -53 * 1.01 + 2.0 ** -47) * ref
    runs = []
    for _ in range(4):
        hi, lo = gpu_weighted(d, w, tile, with_lo=True)
        runs.append((hi, hi.astype(np.float64) + lo.astype(np.float64)))
    for hi, pair in runs:
        assert np.all(np.abs(pair - ref) <= bound), "a run leaves the fp64 bound of the exact sum"
    for hi, pair in runs[1:]:
        diff = np.abs(pair - runs[0][1])
        assert np.all(diff <= bound), f"run-to-run difference {diff.max():.3e} beyond the bound"
        # float32 outputs: equal, except that two runs whose fp64 sums straddle
        # a float32 rounding boundary give adjacent floats, the boundary (their
        # midpoint) then lying within the bound of either sum
        ne = hi != runs[0][0]
        if ne.any():
            a, b = hi[ne].astype(np.float64), runs[0][0][ne].astype(np.float64)
            assert np.all(np.nextafter(hi[ne], runs[0][0][ne]) == runs[0][0][ne]), "not adjacent floats"
            assert np.all(np.abs(pair[ne] - (a + b) / 2) <= bound[ne])


# ----------------------------------------------------------------- backward

@pytest.mark.parametrize("tile", [32, 64])
def test_backward_c0_positive(tile):
    d = oracle.flowdirs(demgen.config_dem("c0"))
    g = demgen.lognormal_f32(d.shape, 31)
    assert_rel(gpu_backward(d, g, tile), oracle.backward_f64(d, g), 1e-6, "backward")


def test_backward_signed_bound():
    d = oracle.flowdirs(demgen.fbm_dem(300, 280, sigma=5.0, seed=4))
    g = np.random.default_rng(5).standard_normal(d.shape).astype(np.float32)
    ref = oracle.backward_f64(d, g)
    refabs = oracle.backward_f64(d, np.abs(g))
    got = gpu_backward(d, g, 32).astype(np.float64)
    # error bound for signed sums: 1e-6 relative plus a tiny multiple of sum |terms|
    # (the final float32 rounding contributes 2^-24 |result|)
    assert (np.abs(got - ref) <= 1e-6 * np.abs(ref) + 2.0 ** -40 * refabs + 1e-30).all()


@pytest.mark.parametrize("shape", [(1, 1), (1, 77), (77, 1), (130, 257), (256, 256)])
def test_backward_shapes_and_serpentine(shape):
    if shape == (256, 256):
        d = oracle.flowdirs(demgen.serpentine(*shape))
    else:
        d = oracle.flowdirs(random_dem(*shape, 11, 0.05))
    g = demgen.lognormal_f32(shape, 12)
    for t in (32, 64):
        assert_rel(gpu_backward(d, g, t), oracle.backward_f64(d, g), 1e-6, "backward")


def test_adjoint_dot_identity_gpu():
    d = oracle.flowdirs(demgen.fbm_dem(400, 400, sigma=5.0, seed=12))
    w = demgen.lognormal_f32(d.shape, 13)
    g = demgen.lognormal_f32(d.shape, 14)
    A = gpu_weighted(d, w).astype(np.float64)
    G = gpu_backward(d, g).astype(np.float64)
    lhs = float((g.astype(np.float64) * A).sum())
    rhs = float((G * w.astype(np.float64)).sum())
    assert abs(lhs - rhs) <= 1e-6 * abs(lhs)


def test_autograd_function():
    d = oracle.flowdirs(demgen.fbm_dem(128, 160, sigma=5.0, seed=21))
    w = demgen.lognormal_f32(d.shape, 22)
    wt = to_dev(w).requires_grad_(True)
    A = d8.D8Accum.apply(to_dev(d), wt)
    gauges = torch.tensor([5, 77, 1000, 20000], device=dev())
    loss = (A.reshape(-1)[gauges] ** 2).sum()
    loss.backward()
    Aref = oracle.accum_f64(d, w)
    gout = np.zeros(d.size)
    gout[gauges.cpu().numpy()] = 2 * Aref.reshape(-1)[gauges.cpu().numpy()]
    ref = oracle.backward_f64(d, gout.reshape(d.shape))
    assert_rel(to_np(wt.grad), ref, 1e-6, "autograd")


# ------------------------------------------------------------------- errors

def _status_after(dirs, tile=32, weighted=False):
    ws = d8.workspace(d8.workspace_bytes(*dirs.shape, tile), dev())
    if weighted:
        d8.accum(to_dev(dirs), to_dev(np.ones(dirs.shape, np.float32)), tile=tile, ws=ws)
    else:
        d8.accum(to_dev(dirs), tile=tile, ws=ws)
    return d8.device_status(ws)


@pytest.mark.parametrize("weighted", [False, True])
def test_device_errors(weighted):
    base = np.full((70, 70), 8, np.uint8)
    d = base.copy()
    d[10, 10], d[10, 11] = 0, 4                 # two-cell cycle inside a tile
    assert _status_after(d, weighted=weighted) == d8.D8_ECYCLE
    d = base.copy()
    d[31, 20], d[32, 20] = 6, 2                 # two-cell cycle across a tile edge (tile 32)
    assert _status_after(d, weighted=weighted) == d8.D8_ECYCLE
    d = base.copy()
    d[5, 5] = 9                                 # not a code
    assert _status_after(d, weighted=weighted) == d8.D8_EBADDIR
    d = base.copy()
    d[0, 5] = 2                                 # north off the grid
    assert _status_after(d, weighted=weighted) == d8.D8_EBADDIR
    d = base.copy()
    d[5, 5], d[5, 6] = 0, 255                   # into NoData
    assert _status_after(d, weighted=weighted) == d8.D8_EBADDIR
    assert _status_after(base, weighted=weighted) == d8.D8_OK


def test_backward_device_errors():
    d = np.full((70, 70), 8, np.uint8)
    d[31, 40], d[32, 40] = 6, 2
    ws = d8.workspace(d8.workspace_bytes(70, 70, 32, backward=True), dev())
    d8.accum_backward(to_dev(d), to_dev(np.ones((70, 70), np.float32)), tile=32, ws=ws)
    assert d8.device_status(ws) == d8.D8_ECYCLE


def test_argument_errors():
    d = to_dev(np.full((8, 8), 8, np.uint8))
    with pytest.raises(d8.D8Error) as e:
        d8.accum(d, tile=48)
    assert e.value.status == d8.D8_EINVAL
    with pytest.raises(d8.D8Error) as e:
        d8.accum(d, to_dev(np.ones((8, 8), np.float32)), tile=128)
    assert e.value.status == d8.D8_EUNSUPPORTED
    small = torch.empty(64, dtype=torch.uint8, device=dev())
    with pytest.raises(d8.D8Error) as e:
        d8.accum(d, ws=small)
    assert e.value.status == d8.D8_ENOMEM


# ------------------------------------------------------------------- batched

def _batch_inputs(n=12, seed=40):
    shapes = [(s[0] // 8 + 1, s[1] // 8 + 3) for s in demgen.batch_shapes(n, seed)]
    dems = [demgen.fbm_dem(r, c, sigma=5.0, seed=100 + i) for i, (r, c) in enumerate(shapes)]
    return shapes, dems


@pytest.mark.parametrize("tile,waves", [(32, 1), (64, 4), (64, 0)])
def test_batched_matches_single(tile, waves):
    shapes, dems = _batch_inputs()
    b = d8.Batch(shapes, dev())
    dem_p = b.pack(dems, torch.float32)
    dirs_p = d8.flowdirs_batched(b, dem_p)
    dirs = [oracle.flowdirs(z) for z in dems]
    for got, ref in zip(b.unpack(dirs_p), dirs):
        np.testing.assert_array_equal(to_np(got), ref)
    counts = d8.accum_batched(b, dirs_p, tile=tile, waves=waves)
    for got, ref in zip(b.unpack(counts), dirs):
        np.testing.assert_array_equal(to_np(got), oracle.accum_u32(ref))
    ws_ = [demgen.lognormal_f32(s, 200 + i) for i, s in enumerate(shapes)]
    gs_ = [demgen.lognormal_f32(s, 300 + i) for i, s in enumerate(shapes)]
    w_p = b.pack(ws_, torch.float32)
    g_p = b.pack(gs_, torch.float32)
    A = d8.accum_batched(b, dirs_p, w_p, tile=tile, waves=waves)
    G = d8.accum_backward_batched(b, dirs_p, g_p, tile=tile, waves=waves)
    for i, (ga, gg) in enumerate(zip(b.unpack(A), b.unpack(G))):
        assert_rel(to_np(ga), oracle.accum_f64(dirs[i], ws_[i]), 1e-6, f"batched fwd {i}")
        assert_rel(to_np(gg), oracle.backward_f64(dirs[i], gs_[i]), 1e-6, f"batched bwd {i}")


# ------------------------------------------- every tile / waves configuration

# every launch shape of the counts tile passes: tile 32 with 1, 2, 4 tiles
# per workgroup; tile 64 walk pass with 1, 2, 4 waves and doubling pass with
# 8, 16 waves (and the defaults); tile 128
CONFIGS = [(32, 0), (32, 1), (32, 2), (32, 4), (64, 0), (64, 1), (64, 2), (64, 4), (64, 8), (64, 16), (128, 0),
           (128, 16)]


@pytest.fixture(scope="module")
def dem2k():
    z = demgen.fbm_dem(2048, 1536, sigma=20.0, seed=1, nodata_frac=0.05, nodata_seed=101)
    d = oracle.flowdirs(z)
    return d, oracle.accum_u32(d)


@pytest.mark.parametrize("tile,waves", CONFIGS)
def test_counts_every_config_2k(dem2k, tile, waves):
    d, ref = dem2k
    H, W = d.shape
    b = d8.Batch([(H, W)], dev())
    out = d8.accum_batched(b, to_dev(d).reshape(-1), tile=tile, waves=waves)
    got = to_np(out).reshape(H, W)
    assert d8.device_status() == d8.D8_OK
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("tile,waves", [(32, 1), (32, 2), (32, 4), (64, 2), (64, 4), (64, 8), (64, 16)])
def test_weighted_and_backward_every_config_2k(dem2k, tile, waves):
    d, _ = dem2k
    H, W = d.shape
    w = demgen.lognormal_f32(d.shape, 77)
    b = d8.Batch([(H, W)], dev())
    dd = to_dev(d).reshape(-1)
    A = d8.accum_batched(b, dd, to_dev(w).reshape(-1), tile=tile, waves=waves)
    assert_rel(to_np(A).reshape(H, W), oracle.accum_f64(d, w), 1e-6, "weighted")
    G = d8.accum_backward_batched(b, dd, to_dev(w).reshape(-1), tile=tile, waves=waves)
    assert_rel(to_np(G).reshape(H, W), oracle.backward_f64(d, w), 1e-6, "backward")


def test_unsupported_launch_shapes_are_refused(dem2k):
    d, _ = dem2k
    H, W = d.shape
    b = d8.Batch([(H, W)], dev())
    dd = to_dev(d).reshape(-1)
    w = torch.ones(H * W, dtype=torch.float32, device=dev())
    for tile, waves, weighted in [(32, 8, False), (32, 16, False), (64, 1, True), (128, 8, False), (64, 3, False)]:
        with pytest.raises(d8.D8Error) as e:
            d8.accum_batched(b, dd, w if weighted else None, tile=tile, waves=waves)
        assert e.value.status == d8.D8_EUNSUPPORTED, (tile, waves, weighted)
    with pytest.raises(d8.D8Error) as e:
        d8.accum_backward_batched(b, dd, w, tile=64, waves=1)
    assert e.value.status == d8.D8_EUNSUPPORTED


# ------------------------------------------------ host-resident (streamed)

@pytest.mark.parametrize("shape,strip,nan", [((300, 257), 64, 0.0), ((300, 257), 128, 0.05), ((129, 70), 64, 0.0),
                                             ((64, 64), 64, 0.0), ((65, 3), 64, 0.0), ((1, 500), 64, 0.0),
                                             ((500, 1), 128, 0.0), ((700, 333), 192, 0.03), ((300, 300), 4096, 0.0)])
def test_streamed_counts_exact(shape, strip, nan):
    """Counts of a host-resident field streamed in row strips equal the
    oracle's (strips of 1, 2, 3 tile rows, ragged last strips, a strip taller
    than the DEM)."""
    z = demgen.fbm_dem(*shape, sigma=5.0, seed=sum(shape) + strip, nodata_frac=nan, nodata_seed=9)
    d = oracle.flowdirs(z)
    host = torch.from_numpy(d).pin_memory()
    got = d8.accum_streamed(host, strip_rows=strip, device=dev())
    assert d8.device_status() == d8.D8_OK
    np.testing.assert_array_equal(got.view(torch.int32).numpy().view(np.uint32), oracle.accum_u32(d))


def test_streamed_pageable_host_memory():
    z = demgen.fbm_dem(200, 230, sigma=5.0, seed=41)
    d = oracle.flowdirs(z)
    got = d8.accum_streamed(torch.from_numpy(d), strip_rows=64, device=dev())
    np.testing.assert_array_equal(got.view(torch.int32).numpy().view(np.uint32), oracle.accum_u32(d))
