"""GPU epsilon fill (the conditioning Sec. 3 assumes) against the oracle, bit
for bit: ragged shapes and tile counts, NoData, plateaus and basins wider
than a tile (many tile rounds), magnitudes where inc falls back to the next
float, signed zeros, and the raw fBm surfaces of the benchmark recipe.  Also
the conditioned chain raw DEM -> fill -> flow directions -> counts."""
import numpy as np
import pytest

import demgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - collected on CPU machines too
    pytest.skip("no GPU", allow_module_level=True)

import paper_1605_05773_amd as d8  # noqa: E402
from gpu_util import to_dev, to_np  # noqa: E402


def say(msg):
    print(f"[fill] {msg}", flush=True)


def check(z, eps=1e-3, what=""):
    say(f"{what} {z.shape} eps={eps}")
    got, rounds = d8.fill(to_dev(z), eps, return_rounds=True)
    got = to_np(got)
    ref = oracle.fill_eps(z, eps)
    bad = got.view(np.uint32) != ref.view(np.uint32)
    assert not bad.any(), (what, int(bad.sum()), np.argwhere(bad)[:5].tolist())
    return got, rounds


def raw_fbm(h, w, seed, sigma=5.0, nan=0.0):
    return demgen.fbm_dem(h, w, sigma=sigma, seed=seed, nodata_frac=nan, nodata_seed=seed + 50, fill=False)


@pytest.mark.parametrize("shape", [(1, 1), (1, 200), (200, 1), (2, 2), (3, 3), (64, 64), (65, 65), (63, 130),
                                   (129, 64), (200, 300)])
def test_shapes(shape):
    rng = np.random.default_rng(sum(shape))
    z = (rng.random(shape) * 3).astype(np.float32)
    check(z, what="uniform noise")


@pytest.mark.parametrize("seed,shape,nan", [(0, (300, 257), 0.0), (1, (513, 190), 0.05), (2, (256, 256), 0.1),
                                            (3, (700, 650), 0.03)])
def test_raw_fbm(seed, shape, nan):
    z = raw_fbm(*shape, seed, nan=nan)
    F, rounds = check(z, what="raw fbm")
    assert rounds >= 2


def test_plateau_wider_than_tiles():
    """A flat 300x420 DEM: interior values climb by eps per cell of Chebyshev
    distance from the boundary, across several tiles."""
    z = np.full((300, 420), np.float32(12.5))
    F, rounds = check(z, what="plateau")
    assert rounds >= 3


def test_basin_spanning_many_tiles():
    """A cone-shaped pit 700 cells across that spills through one low
    boundary cell: the fill front crosses many tiles, in every direction."""
    n = 700
    y, x = np.mgrid[0:n, 0:n].astype(np.float64)
    z = (np.hypot(y - 350, x - 350) * 0.01 + 5).astype(np.float32)
    z[0, :] = 100.0
    z[-1, :] = 100.0
    z[:, 0] = 100.0
    z[:, -1] = 100.0
    z[n // 2, -1] = 1.0
    check(z, what="basin")


@pytest.mark.parametrize("eps", [1e-3, 0.5, 1e-6])
def test_eps_values_and_large_magnitudes(eps):
    z = raw_fbm(200, 230, 9) + np.float32(65536.0)   # 1e-3 is below half an ulp here
    check(z, eps=eps, what="offset 2^16")


def test_signed_zeros_and_negatives():
    rng = np.random.default_rng(5)
    z = (rng.integers(-3, 3, size=(150, 170)) * np.float32(1e-3)).astype(np.float32)
    z[rng.random(z.shape) < 0.2] = np.float32(-0.0)
    check(z, what="signed zeros")


def test_all_nodata_and_nan_fringe():
    z = np.full((70, 90), np.nan, np.float32)
    got = to_np(d8.fill(to_dev(z)))
    assert np.isnan(got).all()
    z = raw_fbm(130, 140, 11)
    z[::7, :] = np.nan
    check(z, what="nan stripes")


def test_conditioned_chain_matches_oracle():
    """Raw c0-recipe surface with NoData -> fill -> flow directions -> counts,
    on the GPU, equals the same chain in the oracle; outlets are exactly the
    seeds (no pits remain)."""
    z = raw_fbm(512, 512, 0, nan=0.03)
    Fg = d8.fill(to_dev(z))
    dg = d8.flowdirs(Fg)
    A = d8.accum(dg)
    F = oracle.fill_eps(z)
    d = oracle.flowdirs(F)
    np.testing.assert_array_equal(to_np(dg), d)
    np.testing.assert_array_equal(to_np(A), oracle.accum_u32(d))
    assert d8.device_status() == d8.D8_OK
    raw_outlets = (oracle.flowdirs(z) == 8).sum()
    assert (d == 8).sum() < raw_outlets


def test_repeat_calls_reuse_workspace():
    z1 = raw_fbm(300, 300, 21)
    z2 = raw_fbm(100, 90, 22)
    check(z1, what="first")
    check(z2, what="second, smaller")
    check(z1, what="first again")
