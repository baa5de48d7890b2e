"""Pins of the oracle's epsilon fill (the conditioning Sec. 3 assumes done
before the method runs: pits raised to the level they drain at, flats given
small elevation changes).

Reading pinned here: seeds are the valid cells on the DEM boundary or next to
NoData and keep their elevation; every other valid cell gets
F(c) = max(z(c), min over valid neighbours n of inc(F(n))), with
inc(x) = fl32(x + eps), or the next float above x when that sum rounds back
to x.  Equivalently F(c) is the minimum over 8-connected paths
c = p0, ..., pk ending at a seed of max_i inc^i(z(p_i)).

No expected value below comes from the oracle's code: they are hand-worked
closed forms (plateaus, a drained bowl, a single pit), a pure-Python
enumeration of every simple path on tiny grids (the path form above), a
plain numpy Jacobi iteration of the fixed-point form from +inf, and
properties that pin the fixed point (idempotence, the D8 field of the
result has outlets only at seeds).
"""
import numpy as np
import pytest

import demgen
import oracle

EPS = np.float32(1e-3)
DRC = [(0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0), (1, 1)]


def inc(x, eps=EPS):
    x = np.float32(x)
    y = np.float32(x + np.float32(eps))
    return y if y > x else np.nextafter(x, np.float32(np.inf), dtype=np.float32)


def inc_k(x, k, eps=EPS):
    x = np.float32(x)
    for _ in range(k):
        x = inc(x, eps)
    return x


def seeds_of(z):
    H, W = z.shape
    s = np.zeros(z.shape, bool)
    for r in range(H):
        for c in range(W):
            if np.isnan(z[r, c]):
                continue
            if r in (0, H - 1) or c in (0, W - 1):
                s[r, c] = True
                continue
            s[r, c] = any(np.isnan(z[r + dr, c + dc]) for dr, dc in DRC)
    return s


def py_paths_fill(z, eps=EPS):
    """The path form by exhaustive search: for every cell, every simple
    8-connected path through valid cells that ends at its first seed."""
    H, W = z.shape
    seed = seeds_of(z)
    out = z.copy()
    for r0 in range(H):
        for c0 in range(W):
            if np.isnan(z[r0, c0]) or seed[r0, c0]:
                continue
            best = [np.float32(np.inf)]

            def walk(r, c, k, cost, seen):
                # cost = max over the path so far of inc^i(z(p_i)); p_k = (r, c)
                if cost >= best[0]:
                    return
                if seed[r, c]:
                    best[0] = cost
                    return
                for dr, dc in DRC:
                    rr, cc = r + dr, c + dc
                    if not (0 <= rr < H and 0 <= cc < W) or np.isnan(z[rr, cc]) or (rr, cc) in seen:
                        continue
                    seen.add((rr, cc))
                    walk(rr, cc, k + 1, max(cost, inc_k(z[rr, cc], k + 1, eps)), seen)
                    seen.discard((rr, cc))

            walk(r0, c0, 0, np.float32(z[r0, c0]), {(r0, c0)})
            out[r0, c0] = best[0]
    return out


def np_jacobi_fill(z, eps=EPS):
    """The fixed-point form iterated from +inf on every non-seed cell."""
    H, W = z.shape
    seed = seeds_of(z)
    valid = ~np.isnan(z)
    F = np.where(seed, z, np.float32(np.inf)).astype(np.float32)
    F[~valid] = np.nan
    for _ in range(4 * H * W + 8):
        P = np.full((H + 2, W + 2), np.inf, np.float32)
        P[1:-1, 1:-1] = np.where(valid, F, np.float32(np.inf))
        m = np.full((H, W), np.inf, np.float32)
        for dr, dc in DRC:
            m = np.minimum(m, P[1 + dr:H + 1 + dr, 1 + dc:W + 1 + dc])
        y = (m + np.float32(eps)).astype(np.float32)
        y = np.where(y > m, y, np.nextafter(m, np.float32(np.inf), dtype=np.float32))
        new = np.where(seed | ~valid, F, np.maximum(z, y))
        if np.array_equal(new, F, equal_nan=True):
            return F
        F = new
    raise AssertionError("no convergence")


def assert_same(a, b):
    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32))


# ------------------------------------------------------------ closed forms

def test_hand_drained_bowl():
    """A 3x3 basin that spills east through a seed of elevation 4: every
    basin cell is raised to inc^k(4), k = its king distance (through the
    basin) to the spill cell."""
    z = np.array([[5, 5, 5, 5, 5],
                  [5, 1, 1, 1, 5],
                  [5, 1, 0, 1, 4],
                  [5, 1, 1, 1, 5],
                  [5, 5, 5, 5, 5]], np.float32)
    k = [[0, 0, 0, 0, 0],
         [0, 3, 2, 1, 0],
         [0, 3, 2, 1, 0],
         [0, 3, 2, 1, 0],
         [0, 0, 0, 0, 0]]
    exp = z.copy()
    for r in range(5):
        for c in range(5):
            if k[r][c]:
                exp[r, c] = inc_k(4.0, k[r][c])
    assert_same(oracle.fill_eps(z, 1e-3), exp)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (6, 1), (2, 2), (5, 5), (7, 12), (16, 9)])
def test_plateau_closed_form(shape):
    """A flat DEM: seeds are the boundary; a cell at Chebyshev distance d from
    the boundary becomes inc^d(z0)."""
    H, W = shape
    z0 = np.float32(3.25)
    z = np.full(shape, z0, np.float32)
    exp = np.empty_like(z)
    for r in range(H):
        for c in range(W):
            exp[r, c] = inc_k(z0, min(r, c, H - 1 - r, W - 1 - c))
    assert_same(oracle.fill_eps(z, 1e-3), exp)


def test_single_pit_in_a_plane():
    """z = r + c (every cell drains by a full unit): nothing changes except a
    single sunk cell, raised to inc of its lowest neighbour."""
    z = np.add.outer(np.arange(9), np.arange(11)).astype(np.float32)
    assert_same(oracle.fill_eps(z, 1e-3), z)
    zp = z.copy()
    zp[4, 6] = -10.0
    exp = z.copy()
    exp[4, 6] = inc(z[3, 5])
    assert_same(oracle.fill_eps(zp, 1e-3), exp)


def test_nodata_lake_makes_seeds():
    """Cells next to NoData are seeds and keep their elevation, so a plateau
    around a NaN hole drains into the hole as well as to the boundary."""
    H = W = 11
    z = np.full((H, W), np.float32(1.0))
    z[5, 5] = np.nan
    exp = np.empty_like(z)
    for r in range(H):
        for c in range(W):
            d = min(r, c, H - 1 - r, W - 1 - c, max(abs(r - 5), abs(c - 5)) - 1)
            exp[r, c] = inc_k(1.0, d)
    exp[5, 5] = np.nan
    got = oracle.fill_eps(z, 1e-3)
    assert np.isnan(got[5, 5])
    m = ~np.isnan(exp)
    assert_same(got[m], exp[m])


def test_increment_below_half_ulp_uses_next_float():
    """At 2^16 an eps of 1e-3 is below half an ulp, so inc is the next float."""
    z = np.full((3, 3), np.float32(65536.0))
    got = oracle.fill_eps(z, 1e-3)
    assert got[1, 1] == np.nextafter(np.float32(65536.0), np.float32(np.inf), dtype=np.float32)
    assert got[1, 1] > z[1, 1]


# --------------------------------------- exhaustive paths, Jacobi, properties

@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("shape", [(4, 4), (5, 5), (4, 6), (3, 7)])
def test_matches_path_enumeration(seed, shape):
    rng = np.random.default_rng(seed)
    z = rng.integers(0, 6, size=shape).astype(np.float32) * np.float32(0.5)
    if seed % 3 == 2:
        z[rng.integers(0, shape[0]), rng.integers(0, shape[1])] = np.nan
    assert_same(oracle.fill_eps(z, 1e-3), py_paths_fill(z))


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("shape,nan", [((9, 9), 0.0), ((13, 21), 0.05), ((30, 17), 0.1), ((1, 12), 0.0)])
def test_matches_numpy_jacobi(seed, shape, nan):
    rng = np.random.default_rng(100 + seed)
    z = (rng.random(shape) * 4).astype(np.float32)
    z[rng.random(shape) < nan] = np.nan
    assert_same(oracle.fill_eps(z, 1e-3), np_jacobi_fill(z))


@pytest.mark.parametrize("eps", [1e-3, 0.25])
def test_raw_fbm_properties(eps):
    """On a raw (unfilled) fBm surface with NoData disks: F >= z, seeds keep z,
    filling again changes nothing, lowest-of-eight on F has outlets exactly at
    the seeds (no pits, no flats), and it matches the Jacobi iteration."""
    z = demgen.fbm_dem(96, 80, sigma=5.0, seed=7, nodata_frac=0.05, nodata_seed=8, fill=False)
    assert (oracle.flowdirs(z) == 8).sum() > (seeds_of(z)).sum()  # the raw surface has pits
    F = oracle.fill_eps(z, eps)
    v = ~np.isnan(z)
    assert np.array_equal(np.isnan(F), ~v)
    assert (F[v] >= z[v]).all()
    s = seeds_of(z)
    assert_same(F[s], z[s])
    assert_same(oracle.fill_eps(F, eps), F)
    d = oracle.flowdirs(F)
    assert np.array_equal(d == 8, s)
    assert_same(F, np_jacobi_fill(z, np.float32(eps)))
    assert (F[v] > z[v]).any()


def test_signed_zero_is_below_positive_zero():
    """Ties between -0 and +0 follow the total order of the bit patterns: a
    cell at -0 next to a seed at -eps is raised to inc(-eps) = +0."""
    e = np.float32(1e-3)
    z = np.full((3, 4), np.float32(5.0))
    z[1, 0] = -e
    z[1, 1] = np.float32(-0.0)
    got = oracle.fill_eps(z, 1e-3)
    assert got[1, 1].view(np.uint32) == np.float32(0.0).view(np.uint32)
    assert got[1, 0] == -e
