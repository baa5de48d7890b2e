"""GPU parity at the benchmark sizes, in the launch configuration bench.py times
(default tile and waves).

Where the oracle finishes in seconds (8192^2 with NoData, 4096^2 weighted, the
512-DEM batch) the GPU results are compared with it cell by cell.  At 32768^2
and on the 16384^2 serpentine they are checked by properties that hold at any
size and pin the result completely: on a D8 forest the recursion of Eq. (1),
A(p) = w(p) + sum of A over the cells draining into p, has exactly one
solution, so an exact integer check of it at every cell (done here with plain
torch integer ops, independent of the library) proves the counts; the
serpentine adds its closed forms; flow directions are compared with the
oracle on sampled row bands.
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
from gpu_util import assert_rel, dev, to_dev, to_np  # noqa: E402

DR = [0, -1, -1, -1, 0, 1, 1, 1]
DC = [1, 1, 0, -1, -1, -1, 0, 1]


def say(msg):
    print(f"[fullsize] {msg}", flush=True)


def identity_mismatches(dirs_t, A_t):
    """Cells where A != [valid] + sum of A over the cells draining in (int64,
    on the GPU with torch), plus NoData cells with A != 0."""
    H, W = dirs_t.shape
    A = A_t.to(torch.int64) if A_t.dtype != torch.uint32 else A_t.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    S = torch.zeros((H + 2, W + 2), dtype=torch.int64, device=A.device)
    for k in range(8):
        contrib = torch.where(dirs_t == k, A, torch.zeros((), dtype=torch.int64, device=A.device))
        S[1 + DR[k]:H + 1 + DR[k], 1 + DC[k]:W + 1 + DC[k]] += contrib
        del contrib
    valid = (dirs_t != 255).to(torch.int64)
    bad = (A != valid + S[1:H + 1, 1:W + 1]).sum().item()
    del S
    return bad, A


def outlet_total(dirs_t, A64):
    return A64[dirs_t == 8].sum().item()


def rows_vs_oracle(z_t, dirs_t, nbands=4, rows=64, seed=0):
    """Flow directions of sampled row bands against the oracle (a band plus a
    one-row halo; its own first/last row are not compared)."""
    H, W = z_t.shape
    rng = np.random.default_rng(seed)
    starts = [0, H - rows] + list(rng.integers(1, H - rows - 1, nbands))
    for r0 in starts:
        lo, hi = max(r0 - 1, 0), min(r0 + rows + 1, H)
        zb = z_t[lo:hi].cpu().numpy()
        ref = oracle.flowdirs(zb)
        got = dirs_t[lo:hi].cpu().numpy()
        a = 1 if lo > 0 else 0
        b = (hi - lo) - (1 if hi < H else 0)
        np.testing.assert_array_equal(got[a:b], ref[a:b], err_msg=f"band at row {r0}")


# ------------------------------------------------------- 32768^2, one GPU

def test_counts_32768_identity():
    """The bench's size and configuration on a rough tilted surface with NoData
    holes (every interior path meanders towards the north-west corner, so the
    perimeter forest is as deep as the grid)."""
    n = 32768
    g = torch.Generator(device=dev()).manual_seed(2)
    say("generating 32768^2 surface on the GPU")
    y = torch.arange(n, device=dev(), dtype=torch.float32).view(n, 1)
    x = torch.arange(n, device=dev(), dtype=torch.float32).view(1, n)
    z = 0.01 * (x + y) + 0.008 * torch.rand((n, n), generator=g, device=dev())
    z[torch.rand((n, n), generator=g, device=dev()) < 1e-4] = float("nan")
    del x, y
    dirs = d8.flowdirs(z)
    torch.cuda.synchronize()
    say("flow directions: sampled bands vs oracle")
    rows_vs_oracle(z, dirs)
    say("accumulating")
    A = d8.accum(dirs)
    torch.cuda.synchronize()
    assert d8.device_status() == d8.D8_OK
    say("identity check")
    bad, A64 = identity_mismatches(dirs, A)
    assert bad == 0
    assert outlet_total(dirs, A64) == (dirs != 255).sum().item()
    del A64
    say("fused DEM -> counts equals flowdirs + accum")
    A2, dirs2 = d8.accum_dem(z)
    torch.cuda.synchronize()
    assert d8.device_status() == d8.D8_OK
    assert torch.equal(dirs2, dirs)
    assert torch.equal(A2.view(torch.int32), A.view(torch.int32))


@pytest.mark.timeout(900)
def test_counts_c2a_workload_exact():
    """The benchmarked workload itself: the 32768^2 fBm DEM (sigma 50 m,
    Hurst 0.7, tilt 0.01, eps-filled), default tile, as bench.py times it.
    Flow directions and counts are compared with the oracle at every cell,
    and the recursion identity and the outlet total are checked on the GPU."""
    say("c2a: generating (or loading) the 32768^2 DEM")
    z = demgen.config_dem("c2a")
    zt = to_dev(z)
    dirs = d8.flowdirs(zt)
    del zt
    say("c2a: accumulating (default tile)")
    A = d8.accum(dirs)
    torch.cuda.synchronize()
    assert d8.device_status() == d8.D8_OK
    say("c2a: identity check")
    bad, A64 = identity_mismatches(dirs, A)
    assert bad == 0
    assert outlet_total(dirs, A64) == dirs.numel()
    del A64
    torch.cuda.empty_cache()
    say("c2a: oracle flow directions")
    dref = oracle.flowdirs(z)
    del z
    np.testing.assert_array_equal(to_np(dirs), dref)
    say("c2a: oracle counts")
    ref = oracle.accum_u32(dref)
    assert np.array_equal(to_np(A), ref)


def test_counts_serpentine_16384_closed_forms():
    n = 16384
    say("serpentine 16384^2")
    z = to_dev(demgen.serpentine_fast(n, n))
    dirs = d8.flowdirs(z)
    del z
    A = d8.accum(dirs)
    torch.cuda.synchronize()
    assert d8.device_status() == d8.D8_OK
    bad, A64 = identity_mismatches(dirs, A)
    assert bad == 0
    edge = torch.zeros((n, n), dtype=torch.bool, device=dev())
    edge[0] = edge[-1] = True
    edge[:, 0] = edge[:, -1] = True
    assert A64.max().item() == n * n - (4 * n - 5)
    assert (A64[edge] == 1).sum().item() == 4 * n - 5


# ---------------------------------------------- 8192^2 with NoData (oracle)

@pytest.fixture(scope="module")
def c1():
    z = demgen.config_dem("c1")
    d = oracle.flowdirs(z)
    return z, d


def test_c1_flowdirs_and_counts_exact(c1):
    z, d = c1
    dd = d8.flowdirs(to_dev(z))
    np.testing.assert_array_equal(to_np(dd), d)
    got = to_np(d8.accum(dd))
    assert d8.device_status() == d8.D8_OK
    np.testing.assert_array_equal(got, oracle.accum_u32(d))


def test_c1_streamed_exact(c1):
    """The 8192^2 field with NoData held in pinned host memory, streamed in
    strips of 1024 rows: counts equal the oracle's."""
    _, d = c1
    got = d8.accum_streamed(torch.from_numpy(d).pin_memory(), strip_rows=1024, device=dev())
    assert d8.device_status() == d8.D8_OK
    np.testing.assert_array_equal(got.view(torch.int32).numpy().view(np.uint32), oracle.accum_u32(d))


def test_c1_weighted_and_backward(c1):
    _, d = c1
    w = demgen.lognormal_f32(d.shape, 303)
    g = demgen.lognormal_f32(d.shape, 304)
    dd = to_dev(d)
    A = to_np(d8.accum(dd, to_dev(w)))
    assert_rel(A, oracle.accum_f64(d, w), 1e-6, "c1 weighted")
    G = to_np(d8.accum_backward(dd, to_dev(g)))
    assert d8.device_status() == d8.D8_OK
    assert_rel(G, oracle.backward_f64(d, g), 1e-6, "c1 backward")


# ----------------------------------- 4096^2 weighted: gauges, targets, FD

def test_c3_gauges_targets_and_finite_differences():
    """Forward vs fp64; the gradient of L = sum over 64 gauges of (A - t)^2 vs
    the fp64 adjoint; 32 central differences of L (exact for a quadratic, so
    any step works; h = 1) on the fp64 oracle vs the GPU gradient."""
    z = demgen.config_dem("c3")
    d = oracle.flowdirs(z)
    w = demgen.lognormal_f32(d.shape, 303)
    xi = demgen.normal_f64(d.shape, 304)
    Aw = oracle.accum_f64(d, w)
    cnt = oracle.accum_u32(d)
    rng = np.random.default_rng(305)
    cand = np.flatnonzero(cnt.ravel() >= 1000)
    gauges = rng.choice(cand, 64, replace=False)
    t = oracle.accum_f64(d, (w.astype(np.float64) * np.exp(0.2 * xi)))
    tg = t.ravel()[gauges]

    dd = to_dev(d)
    out = torch.empty(d.shape, dtype=torch.float32, device=dev())
    lo = torch.empty(d.shape, dtype=torch.float32, device=dev())
    d8.accum(dd, to_dev(w), out=out, out_lo=lo)
    A_gpu = to_np(out)
    assert_rel(A_gpu, Aw, 1e-6, "c3 forward")
    # residuals from (out, out_lo): RN32(sum) and RN32(sum - out) of the fp64 sum
    Ag = to_np(out).astype(np.float64).ravel()[gauges] + to_np(lo).astype(np.float64).ravel()[gauges]
    resid = Ag - tg
    gL = np.zeros(d.size, np.float64)
    gL[gauges] = 2.0 * resid
    g32 = gL.astype(np.float32).reshape(d.shape)
    G_gpu = to_np(d8.accum_backward(dd, to_dev(g32)))
    assert d8.device_status() == d8.D8_OK
    G_ref = oracle.backward_f64(d, g32)
    nz = G_ref != 0
    assert (G_gpu[~nz] == 0).all()
    assert_rel(G_gpu[nz], G_ref[nz], 1e-6, "c3 backward")

    # finite differences on the fp64 oracle
    def loss(wv):
        a = oracle.accum_f64(d, wv).ravel()[gauges]
        return float(((a - tg) ** 2).sum())

    up = np.flatnonzero(G_ref.ravel() != 0)
    fd_cells = np.random.default_rng(306).choice(up, 32, replace=False)
    w64 = w.astype(np.float64)
    for c in fd_cells:
        wp = w64.copy()
        wp.ravel()[c] += 1.0
        wm = w64.copy()
        wm.ravel()[c] -= 1.0
        fd = (loss(wp) - loss(wm)) / 2.0
        an = float(G_gpu.ravel()[c])
        assert abs(an - fd) <= 1e-5 * abs(fd) + 1e-9, (c, an, fd)


# ------------------------------------------------------ 512-DEM batch

def test_c4_batch_vs_oracle():
    say("generating the 512-DEM batch")
    shapes, dems, ws, gs = demgen.c4_batch()
    b = d8.Batch(shapes, dev())
    dirs = [oracle.flowdirs(z) for z in dems]
    dp = b.pack([to_dev(x) for x in dirs], torch.uint8)
    wp = b.pack([to_dev(x) for x in ws], torch.float32)
    gp = b.pack([to_dev(x) for x in gs], torch.float32)
    say("batched calls")
    C = b.unpack(d8.accum_batched(b, dp))
    A = b.unpack(d8.accum_batched(b, dp, wp))
    G = b.unpack(d8.accum_backward_batched(b, dp, gp))
    assert d8.device_status() == d8.D8_OK
    for i in range(len(shapes)):
        np.testing.assert_array_equal(to_np(C[i]), oracle.accum_u32(dirs[i]), err_msg=f"dem {i}")
        assert_rel(to_np(A[i]), oracle.accum_f64(dirs[i], ws[i]), 1e-6, f"batched weighted {i}")
        assert_rel(to_np(G[i]), oracle.backward_f64(dirs[i], gs[i]), 1e-6, f"batched backward {i}")


# --------------------------------------------- conditioning at 8192^2 (oracle)

def test_c1_raw_fill_exact():
    """The 8192^2 surface with NoData disks before conditioning: the GPU fill
    equals the oracle bit for bit, and lowest-of-eight on it leaves outlets
    only on the DEM boundary and next to NoData."""
    say("raw c1 surface")
    z = demgen.config_dem("c1", raw=True)
    say("GPU fill")
    Fg, rounds = d8.fill(to_dev(z), 1e-3, return_rounds=True)
    say(f"rounds {rounds}; oracle fill")
    F = oracle.fill_eps(z, 1e-3)
    got = to_np(Fg)
    assert np.array_equal(got.view(np.uint32), F.view(np.uint32))
    dg = to_np(d8.flowdirs(Fg))
    seeds = ~np.isnan(z)
    inner = np.zeros_like(seeds)
    inner[1:-1, 1:-1] = True
    nan = np.isnan(z)
    near = nan.copy()
    for dr in (-1, 0, 1):
        for dc in (-1, 0, 1):
            near |= np.roll(np.roll(nan, dr, 0), dc, 1)
    seeds &= ~inner | near
    assert np.array_equal(dg == 8, seeds)


# ------------------------------------------------- the largest shape accepted

def identity_mismatches_chunked(dirs_t, A_t, rows=4096):
    """identity_mismatches in row bands with a one-row halo (bounded memory)."""
    H, W = dirs_t.shape
    bad, outlet = 0, 0
    for r0 in range(0, H, rows):
        r1 = min(H, r0 + rows)
        lo, hi = max(0, r0 - 1), min(H, r1 + 1)
        d = dirs_t[lo:hi]
        A = A_t[lo:hi].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        S = torch.zeros((hi - lo + 2, W + 2), dtype=torch.int64, device=A.device)
        for k in range(8):
            S[1 + DR[k]:hi - lo + 1 + DR[k], 1 + DC[k]:W + 1 + DC[k]] += torch.where(
                d == k, A, torch.zeros((), dtype=torch.int64, device=A.device))
        a, b = r0 - lo, r1 - lo
        valid = (d[a:b] != 255).to(torch.int64)
        bad += (A[a:b] != valid + S[1 + a:1 + b, 1:W + 1]).sum().item()
        outlet += A[a:b][d[a:b] == 8].sum().item()
        del S, A
    return bad, outlet


def test_counts_largest_shape_identity():
    """rows * cols = 2^32 - 1, the largest grid the library accepts (uint32
    counts and cell numbering): a tilted rough surface with NoData holes,
    checked by the recursion identity at every cell and the outlet total."""
    H, W = 65535, 65537
    assert H * W == (1 << 32) - 1
    say(f"largest shape {H}x{W}: surface")
    g = torch.Generator(device=dev()).manual_seed(7)
    z = torch.rand((H, W), generator=g, device=dev())
    z.mul_(0.008)
    z.add_(torch.arange(H, device=dev(), dtype=torch.float32).view(H, 1) * 0.01)
    z.add_(torch.arange(W, device=dev(), dtype=torch.float32).view(1, W) * 0.01)
    holes = torch.rand((H, W), generator=g, device=dev()) < 2e-6
    z[holes] = float("nan")
    del holes
    dirs = d8.flowdirs(z)
    nvalid = (dirs != 255).sum().item()
    del z
    torch.cuda.empty_cache()
    say("accumulating")
    A = d8.accum(dirs)
    torch.cuda.synchronize()
    assert d8.device_status() == d8.D8_OK
    d8._ws_cache.clear()
    torch.cuda.empty_cache()
    say("identity check in bands")
    bad, outlet = identity_mismatches_chunked(dirs, A)
    assert bad == 0
    assert outlet == nvalid


# ------------------------------------------ conditioning at 32768^2 (properties)

def _keys(f):
    """Order-preserving int64 keys of float32 values (-0 below +0)."""
    b = f.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    return torch.where(b >= 0x80000000, b ^ 0xFFFFFFFF, b | 0x80000000)


def _unkey(k):
    b = torch.where(k >= 0x80000000, k & 0x7FFFFFFF, k ^ 0xFFFFFFFF)
    return (b - ((b >> 31) << 32)).to(torch.int32).view(torch.float32)


def test_fill_32768_fixed_point():
    """A 32768^2 tilted surface whose noise exceeds the tilt (pits and small
    depressions everywhere) with NoData holes: the GPU fill satisfies the
    defining equations at every cell, which have exactly one solution --
    seeds keep z, every other valid cell equals max(z, min over valid
    neighbours of inc(F)) in the total order of the float bits -- and
    lowest-of-eight on it has outlets exactly at the seeds."""
    n = 32768
    eps = np.float32(1e-3)
    g = torch.Generator(device=dev()).manual_seed(11)
    say("fill 32768^2: surface")
    z = torch.rand((n, n), generator=g, device=dev()).mul_(0.05)
    z.add_(torch.arange(n, device=dev(), dtype=torch.float32).view(n, 1) * 0.01)
    z.add_(torch.arange(n, device=dev(), dtype=torch.float32).view(1, n) * 0.01)
    z[torch.rand((n, n), generator=g, device=dev()) < 2e-6] = float("nan")
    say("GPU fill")
    F, rounds = d8.fill(z, float(eps), return_rounds=True)
    say(f"{rounds} rounds; checking the equations in bands")
    d8._ws_cache.clear()
    torch.cuda.empty_cache()
    inf_key = int(_keys(torch.tensor([float("inf")], device=dev()))[0])
    rows = 2048
    for r0 in range(0, n, rows):
        r1 = min(n, r0 + rows)
        lo, hi = max(0, r0 - 1), min(n, r1 + 1)
        zb, Fb = z[lo:hi], F[lo:hi]
        assert torch.equal(torch.isnan(zb), torch.isnan(Fb))
        K = torch.full((hi - lo + 2, n + 2), inf_key, dtype=torch.int64, device=dev())
        kf = _keys(Fb)
        K[1:-1, 1:-1] = torch.where(torch.isnan(Fb), torch.full_like(kf, inf_key), kf)
        a, b = r0 - lo, r1 - lo
        m = torch.full((b - a, n), inf_key, dtype=torch.int64, device=dev())
        nanadj = torch.zeros((b - a, n), dtype=torch.bool, device=dev())
        Zp = torch.full((hi - lo + 2, n + 2), float("nan"), device=dev())
        Zp[1:-1, 1:-1] = zb
        for dr, dc in zip(DR, DC):
            m = torch.minimum(m, K[1 + a + dr:1 + b + dr, 1 + dc:n + 1 + dc])
            nanadj |= torch.isnan(Zp[1 + a + dr:1 + b + dr, 1 + dc:n + 1 + dc])
        del K, Zp
        mv = _unkey(m)
        y = mv + torch.tensor(eps, device=dev())
        y = torch.where(y > mv, y, torch.nextafter(mv, torch.tensor(float("inf"), device=dev())))
        zc, Fc = zb[a:b], Fb[a:b]
        expect = _unkey(torch.maximum(_keys(zc), _keys(y)))
        rr = torch.arange(r0, r1, device=dev()).view(-1, 1)
        cc = torch.arange(n, device=dev()).view(1, -1)
        seed = (rr == 0) | (rr == n - 1) | (cc == 0) | (cc == n - 1) | nanadj
        valid = ~torch.isnan(zc)
        want = torch.where(seed, zc, expect)
        bad = valid & (want.view(torch.int32) != Fc.view(torch.int32))
        assert not bad.any(), (r0, int(bad.sum()))
    say("outlets of the filled surface")
    dirs = d8.flowdirs(F)
    valid = ~torch.isnan(z)
    P = torch.zeros((n + 2, n + 2), dtype=torch.bool, device=dev())
    P[1:-1, 1:-1] = torch.isnan(z)
    nanadj = torch.zeros_like(valid)
    for dr, dc in zip(DR, DC):
        nanadj |= P[1 + dr:n + 1 + dr, 1 + dc:n + 1 + dc]
    del P
    edge = torch.zeros_like(valid)
    edge[0] = edge[-1] = True
    edge[:, 0] = edge[:, -1] = True
    seeds = valid & (edge | nanadj)
    assert torch.equal(dirs == 8, seeds)
