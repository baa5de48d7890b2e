"""Benchmark: D8 up-slope area (flow accumulation) throughput on one MI355X.

One step = one d8_accum call (tile pass with unknown inflows -> perimeter
resolve -> final tile pass) over the resident direction field of the
workload, unit weights, uint32 counts.  Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2a]

Default workload: a 32768 x 32768 synthetic DEM (1.07 G cells; fBm sigma
50 m, Hurst 0.7, tilt 0.01, eps-filled), the size the throughput target is
stated for.  Inputs are generated on the host once (cached under
$D8_CACHE), copied to HBM and converted to directions with d8_flowdirs
before the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcells/s D8 accumulation + % HBM roofline; fwd+bwd vs plain fwd Gcells/s"
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell of each kernel phase (minimal model):
#   count_tile_emit  : 1 B direction in + 4 B tile-local count out
#   count_tile_final : 1 B direction in (the read-modify-write of the cells
#                      downstream of receivers depends on the data)
#   flowdirs         : 4 B elevation in + 1 B direction out
ALG_BYTES_PER_CELL = {"count_tile_emit": 5.0, "count_tile_final": 1.0, "flowdirs": 5.0,
                      "weighted_tile_final": 9.0, "weighted_tile_emit": 5.0,
                      "backward_tile_final": 9.0, "backward_tile_emit": 5.0}
OP_BYTES_PER_CELL = 5.0  # d8_accum counts: 1 B direction in + 4 B count out

WORKLOADS = {
    "c2a": "32768x32768 fBm DEM (sigma 50 m, Hurst 0.7, tilt 0.01, eps-filled 1e-3), unit weights, uint32 counts",
    "c1": "8192x8192 fBm DEM (sigma 20 m) with ~5% NoData disks r=8..64, unit weights, uint32 counts",
    "c2b": "16384x16384 walled serpentine DEM (one boustrophedon channel), unit weights, uint32 counts",
    "c0": "512x512 fBm DEM (sigma 5 m), unit weights, uint32 counts",
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha():
    h = hashlib.sha256()
    for f in ("d8_kernels.hip", "d8_dev.hpp"):
        with open(os.path.join(ROOT, "paper_1605_05773_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(phase, workload, tile):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    rec = t.get(f"{phase}:{workload}:{tile}")
    if not rec or rec.get("kernel_sha") != kernel_source_sha():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(z_full, workload):
    """The oracle (plain single-threaded C Kahn queue) on a bounded sample: the
    top-left quarter of the same DEM, its own flow directions recomputed so the
    crop is a valid field."""
    import oracle

    oracle.build()
    H, W = z_full.shape
    if H * W > (1 << 28):
        h, w = H // 2, W // 2
        sample = f"top-left {h}x{w} crop of the {workload} DEM (flow directions recomputed on the crop)"
        z = np.ascontiguousarray(z_full[:h, :w])
    else:
        h, w = H, W
        sample = f"the full {workload} DEM"
        z = z_full
    d = oracle.flowdirs(z)
    t0 = time.perf_counter()
    oracle.accum_u32(d)
    dt = time.perf_counter() - t0
    return {"value": round(h * w / dt / 1e9, 5), "unit": "Gcells/s", "cores": 1, "kind": "oracle", "sample": sample,
            "seconds": round(dt, 3), "host_nproc": os.cpu_count(), "host_cpu": host_cpu()}


def identity_check(dirs, counts, rows=4096):
    """Cells where counts != [valid] + sum of counts over the cells draining in,
    and the sum of counts over outlet cells (int64 torch ops on the device, in
    row bands with a one-row halo)."""
    import torch

    dr = (0, -1, -1, -1, 0, 1, 1, 1)
    dc = (1, 1, 0, -1, -1, -1, 0, 1)
    H, W = dirs.shape
    bad, outlet = 0, 0
    for r0 in range(0, H, rows):
        r1 = min(H, r0 + rows)
        lo, hi = max(0, r0 - 1), min(H, r1 + 1)
        d = dirs[lo:hi]
        A = counts[lo:hi].view(torch.int32).to(torch.int64) & 0xFFFFFFFF
        S = torch.zeros((hi - lo + 2, W + 2), dtype=torch.int64, device=A.device)
        zero = torch.zeros((), dtype=torch.int64, device=A.device)
        for k in range(8):
            S[1 + dr[k]:hi - lo + 1 + dr[k], 1 + dc[k]:W + 1 + dc[k]] += torch.where(d == k, A, zero)
        a, b = r0 - lo, r1 - lo
        valid = (d[a:b] != 255).to(torch.int64)
        bad += int((A[a:b] != valid + S[1 + a:1 + b, 1:W + 1]).sum().item())
        outlet += int(A[a:b][d[a:b] == 8].sum().item())
        del S, A
    return bad, outlet


def host_cpu():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2a", choices=sorted(WORKLOADS))
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fwdbwd", action="store_true")
    ap.add_argument("--no-fused", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-fill", action="store_true")
    ap.add_argument("--no-streamed", action="store_true")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 1 GiB device-to-device copy (profiler calibration of byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only (the library runs the whole path on one device); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import demgen
    import paper_1605_05773_amd as d8

    dev = torch.device("cuda", 0)
    t0 = time.time()
    z = demgen.config_dem(args.workload)
    H, W = z.shape
    log(f"workload {args.workload} {H}x{W} ready in {time.time() - t0:.1f}s")
    dem = torch.from_numpy(np.ascontiguousarray(z)).to(dev)
    dirs = d8.flowdirs(dem)
    torch.cuda.synchronize()
    out = torch.empty((H, W), dtype=torch.uint32, device=dev)
    ws = d8.workspace(d8.workspace_bytes(H, W, args.tile), dev)
    stream = torch.cuda.current_stream(dev)

    for _ in range(args.warmup):
        d8.accum(dirs, tile=args.tile, out=out, ws=ws)
    torch.cuda.synchronize()
    st = d8.device_status(ws)
    if st != d8.D8_OK:
        raise SystemExit(f"device status {st} after warmup")
    log(f"warmup done ({args.warmup} steps)")

    # Timed region: exactly `steps` steps, synchronised on both sides.
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        d8.accum(dirs, tile=args.tile, out=out, ws=ws)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    value = H * W / (ms_step * 1e-3) / 1e9
    log(f"timed {args.steps} steps: {ms_step:.3f} ms/step, {value:.1f} Gcells/s (wall {wall:.2f}s)")

    # The timed output, checked once outside the timed region: on a D8 forest
    # the recursion of Eq. (1) has exactly one solution, so an exact integer
    # check at every cell plus the outlet total proves the counts.
    bad, outlet = identity_check(dirs, out)
    nvalid = int((dirs != 255).sum().item())
    if bad or outlet != nvalid:
        raise SystemExit(f"timed output fails the Eq. (1) identity at {bad} cells "
                         f"(outlet total {outlet} vs {nvalid} valid cells)")
    log("timed output verified: Eq. (1) identity at every cell, outlet total = valid cells")

    # Per-step spread: one pair of events around each step (a separate pass).
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev:
        a_.record(stream)
        d8.accum(dirs, tile=args.tile, out=out, ws=ws)
        b_.record(stream)
    torch.cuda.synchronize()
    per_step = sorted(a_.elapsed_time(b_) for a_, b_ in ev)
    step_median, step_min = per_step[len(per_step) // 2], per_step[0]

    # Per-phase durations: the library records HIP events around each kernel
    # phase on the same stream (a separate pass of the same steps).
    d8.phase_timing(True)
    for _ in range(args.steps):
        d8.accum(dirs, tile=args.tile, out=out, ws=ws)
    torch.cuda.synchronize()
    phases = d8.phase_report()
    d8.phase_timing(False)
    phase_ms = {k: round(v[0] / v[1], 4) for k, v in phases.items()}
    log(f"phases (ms/launch): {phase_ms}")
    tile = args.tile or 64  # library default tile side
    dominant = max(phase_ms, key=phase_ms.get)
    cells = H * W
    if dominant in ALG_BYTES_PER_CELL:
        alg = ALG_BYTES_PER_CELL[dominant] * cells
        achieved = alg / (phase_ms[dominant] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(dominant, args.workload, tile), "kernel": dominant,
                "alg_bytes_per_launch": alg}
    else:
        # the resolve: latency-bound rounds over the perimeter graph; reported
        # against HBM with the bytes of its slot arrays touched per round
        roof = {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": measured_traffic(dominant, args.workload, tile), "kernel": dominant}
    op_gbs = OP_BYTES_PER_CELL * cells / (ms_step * 1e-3) / 1e9

    extra = {"verified": True, "verification": "Eq. (1) identity at every cell and outlet total, on the timed output",
             "phase_ms": phase_ms, "step_ms_median": round(step_median, 4), "step_ms_min": round(step_min, 4),
             "op_roofline_frac": round(op_gbs / HBM_PEAK_GBS, 4),
             "op_bytes_per_cell": OP_BYTES_PER_CELL, "wall_s": round(wall, 3)}

    if not args.no_streamed:
        # The same counts with the direction field and the counts in pinned
        # host memory, streamed through the GPU in strips of 2048 rows: the
        # PCIe-inclusive rate (14 B/cell cross the link: 1 + 4 out in the tile
        # pass, 1 + 4 in and 4 out in the finalising pass).
        dh = dirs.cpu().pin_memory()
        oh = torch.empty((H, W), dtype=torch.uint32, pin_memory=True)
        sr = min(2048, (H + 63) // 64 * 64)
        wss = d8.workspace(d8.lib().d8_accum_streamed_workspace_bytes(H, W, sr), dev)
        d8.accum_streamed(dh, strip_rows=sr, out=oh, device=dev, ws=wss)
        ns = 3
        t0 = time.perf_counter()
        for _ in range(ns):
            d8.accum_streamed(dh, strip_rows=sr, out=oh, device=dev, ws=wss)
        st_ms = (time.perf_counter() - t0) * 1e3 / ns
        same = bool(torch.equal(oh.view(torch.int32), out.cpu().view(torch.int32)))
        extra["streamed"] = {"workload": f"{args.workload} direction field and counts in pinned host memory, "
                                         f"strips of {sr} rows", "ms": round(st_ms, 2),
                             "gcells": round(H * W / st_ms / 1e6, 3), "pcie_bytes_per_cell": 14,
                             "pcie_gbs": round(14 * H * W / st_ms / 1e6, 1), "same_as_device": same}
        log(f"streamed: {extra['streamed']}")
        del dh, oh, wss
        d8._ws_cache.clear()
        torch.cuda.empty_cache()

    if not args.no_fused:
        # End to end from the DEM: d8_flowdirs + d8_accum vs the fused
        # d8_accum_dem (codes computed inside the tile pass).
        dtmp = torch.empty_like(dirs)
        for _ in range(2):
            d8.accum_dem(dem, tile=args.tile, out=out, dirs=dtmp, ws=ws)
        torch.cuda.synchronize()
        f0, f1, f2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        f0.record(stream)
        for _ in range(args.steps):
            d8.flowdirs(dem)
            d8.accum(dirs, tile=args.tile, out=out, ws=ws)
        f1.record(stream)
        for _ in range(args.steps):
            d8.accum_dem(dem, tile=args.tile, out=out, dirs=dtmp, ws=ws)
        f2.record(stream)
        torch.cuda.synchronize()
        sep = f0.elapsed_time(f1) / args.steps
        fus = f1.elapsed_time(f2) / args.steps
        extra["dem_to_counts"] = {"separate_ms": round(sep, 4), "fused_ms": round(fus, 4),
                                  "fused_gcells": round(H * W / fus / 1e6, 2),
                                  "separate_gcells": round(H * W / sep / 1e6, 2)}
        log(f"DEM -> counts: {extra['dem_to_counts']}")
        del dtmp
    del dem

    if not args.no_fwdbwd:
        # Forward vs forward+backward of the differentiable weighted form on the
        # 4096^2 workload (lognormal weights, positive upstream gradients).
        zc3 = demgen.config_dem("c3")
        d3 = d8.flowdirs(torch.from_numpy(zc3).to(dev))
        w3 = torch.from_numpy(demgen.lognormal_f32(zc3.shape, 303)).to(dev)
        g3 = torch.from_numpy(demgen.lognormal_f32(zc3.shape, 304)).to(dev)
        o3 = torch.empty(zc3.shape, dtype=torch.float32, device=dev)
        ws3 = torch.empty(d8.workspace_bytes(*zc3.shape, 0, backward=True) + 256, dtype=torch.uint8, device=dev)
        ws3 = ws3[(-ws3.data_ptr()) % 256:]
        for _ in range(2):
            d8.accum(d3, w3, out=o3, ws=ws3)
            d8.accum_backward(d3, g3, ws=ws3)
        torch.cuda.synchronize()
        a0, a1, a2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        a0.record(stream)
        for _ in range(args.steps):
            d8.accum(d3, w3, out=o3, ws=ws3)
        a1.record(stream)
        for _ in range(args.steps):
            d8.accum(d3, w3, out=o3, ws=ws3)
            d8.accum_backward(d3, g3, ws=ws3)
        a2.record(stream)
        torch.cuda.synchronize()
        f_ms = a0.elapsed_time(a1) / args.steps
        fb_ms = a1.elapsed_time(a2) / args.steps
        n3 = zc3.size
        extra["fwd_bwd"] = {"workload": "4096x4096 fBm DEM (sigma 5 m), lognormal(0,1) f32 weights",
                            "fwd_gcells": round(n3 / f_ms / 1e6, 2), "fwd_bwd_gcells": round(n3 / fb_ms / 1e6, 2),
                            "fwd_ms": round(f_ms, 4), "fwd_bwd_ms": round(fb_ms, 4),
                            "ratio": round(f_ms / fb_ms, 4)}
        log(f"fwd/bwd: {extra['fwd_bwd']}")
        del d3, w3, g3, o3, ws3

    if not args.no_batch:
        # The batched differentiable form on the 512-DEM workload (sizes per
        # the log-uniform recipe, lognormal weights and upstream gradients):
        # forward alone vs forward + backward, each replayed as one HIP graph.
        shapes, dems, ws4, gs4 = demgen.c4_batch()
        b = d8.Batch(shapes, dev)
        dp = d8.flowdirs_batched(b, b.pack([torch.from_numpy(x) for x in dems], torch.float32))
        cells4 = b.total
        wp4 = b.pack([torch.from_numpy(x) for x in ws4], torch.float32)
        # the autotuner picks tile side and waves per tile (outside the timing)
        t4, v4, tune_ms = d8.autotune_batched(b, dp, wp4)
        gr = d8.BatchedGraph(b, tile=t4, waves=v4)
        gr.dirs.copy_(dp)
        gr.w.copy_(wp4)
        gr.g.copy_(b.pack([torch.from_numpy(x) for x in gs4], torch.float32))
        gr.capture()
        fwd_graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(fwd_graph):
            d8.accum_batched(b, gr.dirs, gr.w, tile=t4, waves=v4, out=gr.area, ws=gr.ws)
        for _ in range(2):
            fwd_graph.replay()
            gr.replay()
        torch.cuda.synchronize()
        if gr.status() != d8.D8_OK:
            raise SystemExit("device status error in the batched workload")
        c0, c1_, c2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        c0.record(stream)
        for _ in range(args.steps):
            fwd_graph.replay()
        c1_.record(stream)
        for _ in range(args.steps):
            gr.replay()
        c2.record(stream)
        torch.cuda.synchronize()
        bf = c0.elapsed_time(c1_) / args.steps
        bfb = c1_.elapsed_time(c2) / args.steps
        extra["batched_graph"] = {"workload": f"{len(shapes)} DEMs, {cells4} cells (sides log-uniform 64..2048)",
                                  "autotuned": {"tile": t4, "waves": v4, "fwd_bwd_ms": round(tune_ms, 4)},
                                  "fwd_gcells": round(cells4 / bf / 1e6, 2), "fwd_bwd_gcells": round(cells4 / bfb / 1e6, 2),
                                  "fwd_ms": round(bf, 4), "fwd_bwd_ms": round(bfb, 4), "ratio": round(bf / bfb, 4)}
        log(f"batched graph: {extra['batched_graph']}")
        del gr, fwd_graph, dp

    if not args.no_fill:
        # Conditioning before the method: the epsilon fill of the 8192^2 surface
        # with NoData disks, before the generator's own fill (about a quarter
        # of its cells lie in closed depressions).  One call runs tile rounds
        # until nothing changes and synchronises; minimal model 8 B/cell
        # (elevation in, filled elevation out).
        zr = demgen.config_dem("c1", raw=True)
        zr_d = torch.from_numpy(zr).to(dev)
        fo = torch.empty_like(zr_d)
        wsf = d8.workspace(d8.lib().d8_fill_workspace_bytes(*zr.shape), dev)
        _, rounds = d8.fill(zr_d, 1e-3, out=fo, ws=wsf, return_rounds=True)
        torch.cuda.synchronize()
        nf = max(3, args.steps // 4)
        t0 = time.perf_counter()
        for _ in range(nf):
            d8.fill(zr_d, 1e-3, out=fo, ws=wsf)
        torch.cuda.synchronize()
        fill_ms = (time.perf_counter() - t0) * 1e3 / nf
        ncell = zr.size
        gbs = 8.0 * ncell / (fill_ms * 1e-3) / 1e9
        extra["fill"] = {"workload": "8192x8192 fBm (sigma 20 m, Hurst 0.7, tilt 0.01) with ~5% NoData disks, "
                                     "before conditioning; eps 1e-3",
                         "ms": round(fill_ms, 3), "gcells": round(ncell / fill_ms / 1e6, 3), "tile_rounds": rounds,
                         "alg_bytes_per_cell": 8.0, "achieved_gbs": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4)}
        if not args.no_cpu_baseline:
            import oracle

            oracle.build()
            crop = np.ascontiguousarray(zr[:4096, :4096])
            t0 = time.perf_counter()
            oracle.fill_eps(crop, 1e-3)
            dt = time.perf_counter() - t0
            extra["fill"]["cpu_baseline"] = {"value": round(crop.size / dt / 1e9, 5), "unit": "Gcells/s", "cores": 1,
                                             "kind": "oracle", "sample": "top-left 4096x4096 crop of the same surface",
                                             "seconds": round(dt, 3)}
        log(f"fill: {extra['fill']}")
        del zr_d, fo

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        log("calibration copy of 1 GiB done")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(z, args.workload)
        log(f"cpu baseline: {cpu}")

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gcells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "rows": H, "cols": W,
                   "tile": tile, "parallelism": "single-gpu"},
        "roofline": roof, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
