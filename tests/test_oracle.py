"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests reuses the oracle's code to produce an expected value:
expected values come from hand-worked fixtures (tests/golden), closed forms
for planes and the walled serpentine, a pure-Python brute force written from
the physical definition of up-slope area (Sec. 2), and invariants (Eq. 1
itself, the outlet sum, linearity, the adjoint identity).
"""
import math

import numpy as np
import pytest

import demgen
import oracle
from golden_io import load

DRC = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]


# ----------------------------------------------------------- independent helpers

def py_target(dirs, r, c):
    k = int(dirs[r, c])
    if k >= 8:
        return None
    dr, dc = DRC[k]
    return r + dr, c + dc


def py_bruteforce(dirs, w=None):
    """Sec. 2: A(p) is the (weighted) number of cells whose flow passes through p.
    Walk every cell's path and add its weight to each cell on it (pure Python)."""
    H, W = dirs.shape
    A = np.zeros((H, W), dtype=np.float64)
    for r in range(H):
        for c in range(W):
            if dirs[r, c] == 255:
                continue
            wt = 1.0 if w is None else float(w[r, c])
            p, steps = (r, c), 0
            while p is not None:
                A[p] += wt
                p = py_target(dirs, *p)
                steps += 1
                assert steps <= H * W + 1
    return A


def py_pathsum(dirs, g):
    """Gradient of sum(g * A(w)) w.r.t. w(c): the sum of g over every cell that c's
    flow passes through, c included (pure Python walk)."""
    H, W = dirs.shape
    G = np.zeros((H, W), dtype=np.float64)
    for r in range(H):
        for c in range(W):
            if dirs[r, c] == 255:
                continue
            p, s = (r, c), 0.0
            while p is not None:
                s += float(g[p])
                p = py_target(dirs, *p)
            G[r, c] = s
    return G


def random_dem(H, W, seed, nan_frac=0.0):
    rng = np.random.default_rng(seed)
    z = rng.random((H, W)).astype(np.float32)
    if nan_frac:
        z[rng.random((H, W)) < nan_frac] = np.nan
    return z


# ------------------------------------------------------------------ fixtures

@pytest.mark.parametrize("name", ["hand_4x5.txt", "hand_5x5_nodata_tie.txt"])
def test_hand_worked_fixture(name):
    dem, dirs_exp, area_exp = load(name)
    dirs = oracle.flowdirs(dem)
    np.testing.assert_array_equal(dirs, dirs_exp)
    np.testing.assert_array_equal(oracle.accum_u32(dirs), area_exp)
    np.testing.assert_array_equal(oracle.accum_f64(dirs), area_exp.astype(np.float64))
    np.testing.assert_array_equal(oracle.bruteforce_f64(dirs), area_exp.astype(np.float64))


# --------------------------------------------------------- flowdirs closed forms

PLANES = [
    # (a, b) for z = a*x + b*y ; expected interior code (tie order E,NE,N,NW,W,SW,S,SE)
    ((0.01, 0.01), 3),   # NW unique lowest
    ((0.01, 0.0), 3),    # NW, W, SW tie -> NW first
    ((0.0, 0.01), 1),    # NE, N, NW tie -> NE first
    ((-0.01, 0.0), 0),   # E, NE, SE tie -> E first
    ((0.0, -0.01), 5),   # SW, S, SE tie -> SW first
    ((-0.01, -0.01), 7), # SE unique lowest
    ((0.01, -0.01), 5),  # SW unique lowest
    ((-0.01, 0.01), 1),  # NE unique lowest
]


@pytest.mark.parametrize("shape", [(9, 9), (7, 11), (12, 5)])
@pytest.mark.parametrize("plane,code", PLANES)
def test_flowdirs_planes(shape, plane, code):
    H, W = shape
    y, x = np.mgrid[0:H, 0:W].astype(np.float32)
    z = (np.float32(plane[0]) * x + np.float32(plane[1]) * y).astype(np.float32)
    d = oracle.flowdirs(z)
    assert (d[1:-1, 1:-1] == code).all()
    assert (d[0] == 8).all() and (d[-1] == 8).all() and (d[:, 0] == 8).all() and (d[:, -1] == 8).all()


def test_flowdirs_flat_is_outlet():
    d = oracle.flowdirs(np.zeros((6, 6), np.float32))
    assert (d == 8).all()


def test_flowdirs_nodata_rules():
    z = np.arange(49, dtype=np.float32).reshape(7, 7)
    z[3, 3] = np.nan
    d = oracle.flowdirs(z)
    assert d[3, 3] == 255
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            if dr or dc:
                assert d[3 + dr, 3 + dc] == 8
    # cells two away from the hole still drain (this plane falls to the north-west)
    assert d[1, 1] == 3 and d[5, 5] == 3


# ------------------------------------------------------ accumulation closed forms

@pytest.mark.parametrize("shape", [(9, 9), (8, 13), (15, 6)])
def test_accum_plane_closed_form(shape):
    H, W = shape
    y, x = np.mgrid[0:H, 0:W].astype(np.float32)
    z = (np.float32(0.01) * (x + y)).astype(np.float32)
    d = oracle.flowdirs(z)
    A = oracle.accum_u32(d)
    exp = np.ones((H, W), dtype=np.int64)
    for r in range(1, H - 1):
        for c in range(1, W - 1):
            exp[r, c] = 1 + min(H - 2 - r, W - 2 - c)
    for r in range(H):
        for c in range(W):
            if r == 0 or c == 0:
                if 1 <= r + 1 <= H - 2 and 1 <= c + 1 <= W - 2:
                    exp[r, c] = 1 + exp[r + 1, c + 1]
    np.testing.assert_array_equal(A, exp.astype(np.uint32))


@pytest.mark.parametrize("shape", [(16, 16), (12, 20), (10, 9), (9, 10), (7, 7), (40, 33)])
def test_serpentine_closed_forms(shape):
    H, W = shape
    z = demgen.serpentine(H, W)
    d = oracle.flowdirs(z)
    A = oracle.accum_u32(d)
    n = len(range(1, H - 1, 2))          # channel rows
    L = n * (W - 2) + (n - 1)            # path cells
    outlet = A.max()
    # every interior cell drains to the one outlet; every other boundary cell stays 1
    assert outlet == H * W - (2 * H + 2 * W - 5)
    edge = np.zeros((H, W), bool)
    edge[0] = edge[-1] = True
    edge[:, 0] = edge[:, -1] = True
    assert (A[edge] == 1).sum() == 2 * H + 2 * W - 5
    # lowest-of-8 cuts two path cells at each of the n-1 turns; +1 for the outlet cell
    assert oracle.depth(d) == L - 2 * (n - 1) + 1


# --------------------------------------------------------------- brute force pins

@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape,nan", [((1, 1), 0.0), ((1, 9), 0.0), ((9, 1), 0.0), ((2, 2), 0.0),
                                       ((13, 17), 0.0), ((16, 16), 0.15), ((23, 11), 0.3)])
def test_accum_matches_python_bruteforce(seed, shape, nan):
    z = random_dem(*shape, seed=seed, nan_frac=nan)
    d = oracle.flowdirs(z)
    exp = py_bruteforce(d)
    np.testing.assert_array_equal(oracle.accum_u32(d).astype(np.float64), exp)
    np.testing.assert_array_equal(oracle.accum_f64(d), exp)
    np.testing.assert_array_equal(oracle.bruteforce_f64(d), exp)
    w = demgen.lognormal_f32(shape, 500 + seed)
    expw = py_bruteforce(d, w)
    np.testing.assert_allclose(oracle.accum_f64(d, w), expw, rtol=1e-13, atol=0)


@pytest.mark.parametrize("seed", range(4))
def test_accum_filled_fbm_matches_python_bruteforce(seed):
    z = demgen.fbm_dem(24, 31, sigma=5.0, seed=seed)
    d = oracle.flowdirs(z)
    assert (d[1:-1, 1:-1] != 8).all()
    np.testing.assert_array_equal(oracle.accum_u32(d).astype(np.float64), py_bruteforce(d))


def test_serpentine_matches_python_bruteforce():
    d = oracle.flowdirs(demgen.serpentine(12, 14))
    np.testing.assert_array_equal(oracle.accum_u32(d).astype(np.float64), py_bruteforce(d))


# ------------------------------------------------------------------ invariants

def test_c0_identity_outlet_sum_unit_and_linearity():
    z = demgen.config_dem("c0")
    d = oracle.flowdirs(z)
    assert (d[1:-1, 1:-1] != 8).all()  # the fill leaves no interior pit
    A = oracle.accum_u32(d)
    assert np.abs(oracle.identity_residual(d, A)).max() == 0
    assert oracle.outlet_total(d, A) == d.size
    np.testing.assert_array_equal(oracle.accum_f64(d), A.astype(np.float64))
    w1 = demgen.lognormal_f32(d.shape, 1)
    w2 = demgen.lognormal_f32(d.shape, 2)
    A1 = oracle.accum_f64(d, w1)
    A2 = oracle.accum_f64(d, w2)
    assert np.abs(oracle.identity_residual(d, A1, w1)).max() <= 1e-9 * A1.max()
    assert math.isclose(oracle.outlet_total(d, A1), float(w1.astype(np.float64).sum()), rel_tol=1e-12)
    comb = 0.75 * w1.astype(np.float64) - 2.5 * w2.astype(np.float64)
    np.testing.assert_allclose(oracle.accum_f64(d, comb), 0.75 * A1 - 2.5 * A2, rtol=0, atol=1e-9 * A1.max())


def test_c1_like_nodata_identity():
    z = demgen.fbm_dem(300, 257, sigma=20.0, seed=7, nodata_frac=0.05, nodata_seed=9)
    assert 0.05 <= np.isnan(z).mean() < 0.2
    d = oracle.flowdirs(z)
    A = oracle.accum_u32(d)
    assert (A[d == 255] == 0).all()
    assert np.abs(oracle.identity_residual(d, A)).max() == 0
    assert oracle.outlet_total(d, A) == (d != 255).sum()


# -------------------------------------------------------------------- adjoint

@pytest.mark.parametrize("seed", range(4))
def test_backward_matches_python_pathsum(seed):
    z = random_dem(14, 19, seed=seed, nan_frac=0.1 * (seed % 2))
    d = oracle.flowdirs(z)
    g = np.random.default_rng(seed).standard_normal(d.shape).astype(np.float32)
    np.testing.assert_allclose(oracle.backward_f64(d, g), py_pathsum(d, g), rtol=1e-12, atol=1e-12)


def test_backward_dot_identity_and_recursion():
    z = demgen.config_dem("c0")
    d = oracle.flowdirs(z)
    w = demgen.lognormal_f32(d.shape, 11)
    g = demgen.normal_f64(d.shape, 12)
    A = oracle.accum_f64(d, w)
    G = oracle.backward_f64(d, g)
    lhs = float((g * A).sum())
    rhs = float((G * w.astype(np.float64)).sum())
    assert math.isclose(lhs, rhs, rel_tol=1e-12)
    t = oracle.targets(d).reshape(-1)
    Gf, gf = G.reshape(-1), g.reshape(-1)
    down = np.where(t >= 0, Gf[np.maximum(t, 0)], 0.0)
    np.testing.assert_allclose(Gf - down, gf, rtol=0, atol=1e-9 * np.abs(G).max())


def test_finite_difference_exact_for_quadratic_loss():
    # L(w) = sum_g (A_g(w) - t_g)^2 is quadratic in w, so a central difference is exact
    z = demgen.fbm_dem(40, 40, sigma=5.0, seed=3)
    d = oracle.flowdirs(z)
    w = demgen.lognormal_f32(d.shape, 3).astype(np.float64)
    A = oracle.accum_f64(d, w)
    gauges = np.argsort(A.reshape(-1))[-5:]
    tgt = A.reshape(-1)[gauges] * 1.02

    def loss(wv):
        a = oracle.accum_f64(d, wv).reshape(-1)[gauges]
        return float(((a - tgt) ** 2).sum())

    gout = np.zeros(d.size)
    gout[gauges] = 2 * (A.reshape(-1)[gauges] - tgt)
    grad = oracle.backward_f64(d, gout.reshape(d.shape)).reshape(-1)
    for cell in [0, 37, 801, 1200, 1599]:
        e = np.zeros(d.size)
        e[cell] = 1.0
        fd = (loss(w + e.reshape(d.shape)) - loss(w - e.reshape(d.shape))) / 2.0
        assert abs(fd - grad[cell]) <= 1e-9 * max(1.0, abs(grad[cell]))


# ------------------------------------------------------------------- errors

def test_errors_cycle_baddir_offgrid_nodata():
    d = np.full((4, 4), 8, np.uint8)
    d[1, 1], d[1, 2] = 0, 4          # E then W: a two-cell cycle
    for f in (oracle.accum_u32, oracle.accum_f64, oracle.backward_f64):
        with pytest.raises(oracle.OracleError) as e:
            f(d)
        assert e.value.status == oracle.CYCLE
    d = np.full((4, 4), 8, np.uint8)
    d[2, 2] = 9                      # not a direction code
    with pytest.raises(oracle.OracleError) as e:
        oracle.accum_u32(d)
    assert e.value.status == oracle.BADDIR
    d = np.full((4, 4), 8, np.uint8)
    d[0, 1] = 2                      # north off the grid
    with pytest.raises(oracle.OracleError) as e:
        oracle.accum_u32(d)
    assert e.value.status == oracle.BADDIR
    d = np.full((4, 4), 8, np.uint8)
    d[1, 1], d[1, 2] = 0, 255        # into NoData
    with pytest.raises(oracle.OracleError) as e:
        oracle.accum_f64(d)
    assert e.value.status == oracle.BADDIR


# ------------------------------------------------------------------ generator

def test_generator_deterministic_and_filled():
    a = demgen.fbm_dem(64, 80, sigma=5.0, seed=5)
    b = demgen.fbm_dem(64, 80, sigma=5.0, seed=5)
    assert a.tobytes() == b.tobytes()
    d = oracle.flowdirs(a)
    assert (d[1:-1, 1:-1] != 8).all()
    c = demgen.fbm_dem(64, 80, sigma=5.0, seed=6)
    assert a.tobytes() != c.tobytes()


def test_batch_shapes_ranges():
    shapes = demgen.batch_shapes(512, 4)
    assert len(shapes) == 512
    for r, c in shapes:
        lo, hi = min(r, c), max(r, c)
        assert 64 <= hi <= 2048 and lo >= 16
        assert lo == 16 or hi / lo <= 4.0 * (1 + 1.0 / lo)


# ------------------------------------------------- steepest-slope rule (Sec. 3)
# Slope to a neighbour = drop / distance, distance sqrt(2) for diagonals.  On
# a plane z = a*x + b*y (a, b >= 0) the candidate slopes are W: a, N: b,
# NW: (a + b)/sqrt(2), NE: (b - a)/sqrt(2), SW: (a - b)/sqrt(2); the expected
# interior codes below follow from those by hand (margins >= 1 %).

@pytest.mark.parametrize("a,b,lowest,steepest", [
    (0.01, 0.004, 3, 4),    # NW lowest; W steeper (0.01 > 0.014/sqrt2 = 0.0099)
    (0.004, 0.01, 3, 2),    # NW lowest; N steeper
    (0.01, 0.01, 3, 3),     # NW both
    (0.01, 0.0, 3, 4),      # lowest: NW/W/SW tie -> NW; steepest: W (0.01 > 0.0071)
    (0.0, 0.01, 1, 2),      # lowest: NE/N/NW tie -> NE; steepest: N
    (-0.01, 0.004, 1, 0),   # mirrored: NE lowest, E steeper
])
def test_steepest_vs_lowest_planes(a, b, lowest, steepest):
    y, x = np.mgrid[0:20, 0:23].astype(np.float64)
    z = (a * x + b * y).astype(np.float32)
    lo = oracle.flowdirs(z)
    st = oracle.flowdirs(z, rule="steepest")
    assert (lo[1:-1, 1:-1] == lowest).all()
    assert (st[1:-1, 1:-1] == steepest).all()
    assert (st[0] == 8).all() and (st[:, 0] == 8).all() and (st[-1] == 8).all() and (st[:, -1] == 8).all()


def test_steepest_plane_counts_closed_form():
    # a = 0.01, b = 0.004: every interior cell drains W along its row, so an
    # interior cell (r, c) collects the W - 1 - c cells from itself to column
    # W - 2, and the west edge cell collects W - 1.
    H, W = 17, 29
    y, x = np.mgrid[0:H, 0:W].astype(np.float64)
    d = oracle.flowdirs((0.01 * x + 0.004 * y).astype(np.float32), rule="steepest")
    A = oracle.accum_u32(d)
    for r in range(1, H - 1):
        np.testing.assert_array_equal(A[r, 1:W - 1], W - 1 - np.arange(1, W - 1))
        assert A[r, 0] == W - 1 and A[r, W - 1] == 1
    assert (A[0] == 1).all() and (A[-1] == 1).all()


def test_steepest_hand_cases():
    # Centre 10.0 of a 5x5 block (border 100 keeps the other cells out of the
    # way).  Case 1: E drops 1.0 (slope 1.0), NE drops 1.3 (slope 0.919):
    # lowest -> NE (1), steepest -> E (0).  Case 2: no lower neighbour -> 8.
    # Case 3: E and W both drop 1.0 -> first in order: E.  Case 4: NE drops
    # 1.5 (1.0607) beats E 1.0 under both rules.
    def block(e, ne, w=100.0):
        z = np.full((5, 5), 100.0, np.float32)
        z[2, 2] = 10.0
        z[2, 3] = e
        z[1, 3] = ne
        z[2, 1] = w
        return z
    for z, lo, st in [(block(9.0, 8.7), 1, 0), (block(11.0, 12.0), 8, 8), (block(9.0, 50.0, 9.0), 0, 0),
                      (block(9.0, 8.5), 1, 1)]:
        assert oracle.flowdirs(z)[2, 2] == lo
        assert oracle.flowdirs(z, rule="steepest")[2, 2] == st
