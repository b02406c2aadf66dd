#!/usr/bin/env python
"""Frames/s of the forward Gaussian-splatting render on one MI355X.

Workload (default): 3,000,000 Gaussians (256-cluster power-law mixture plus
10% large background Gaussians, SH degree 3, float32 attributes) rendered at
1920x1080 with 16x16 tiles from the default camera; synthetic, seeded.  A step
is one gs_render call -- project, depth sort, tile count/offsets, sorted pair
list, blend -- with the scene already resident in HBM.

Prints ONE JSON line with the frame rate of back-to-back renders, the
per-stage device times (HIP events recorded by the library on the render
stream, from a separate profiled pass), a roofline entry for the dominant
kernel, the frame rate of the BF16 / FP16 attribute-storage variants of the
same frame, and the FP64 oracle's time on a bounded sample of the frame on the
host cores.

    python bench.py [--steps K] [--warmup W] [--variant fp32|bf16|fp16]
                    [--workload C3] [--no-cpu-baseline] [--no-variants]
"""
from __future__ import annotations

import argparse
import functools
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "frames/s and achieved HBM GB/s (% peak), 1080p / 3M Gaussians, FP32 vs BF16 vs batched"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
TILE = 16
# algorithmic FP32 operations of one (pixel, list entry) evaluation of Eq. 1's
# term: offset (2), quadratic form (3 products, 3 conic products, 2 adds,
# 1 scale), exp (1), times opacity (1) = 13; a composited entry adds the
# transmittance update (2) and the weighted colour accumulation (1 + 3 x 2).
FLOPS_EVAL = 13
FLOPS_COMPOSITE = 9
# MI355X FP32 vector peak without packed FP32 (the library is built without
# packed-FP32 instruction selection): 256 CUs x 4 SIMDs x 16 lanes x 2 flops x
# 2.4 GHz
FP32_VECTOR_NONPACKED_TFLOPS = 78.6


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def attr_bytes(dtype: int) -> int:
    return 4 if dtype == 0 else 2


PACKED_RECT_TILES = 255   # views at most this many tiles wide and tall carry packed rectangles through the sort


def algorithmic_bytes(stage: str, n: int, n_vis: int, K: int, R: int, deg: int, dtype: int, W: int, H: int,
                      stats: dict, tuning: dict | None = None) -> float:
    """HBM bytes one frame's launches of a stage must move: each input and
    output once (the per-unit figures below, times the units of the frame).
    ``tuning`` gives the chunk sizes of the binning (count arrays and cursors
    scale with them)."""
    tu = tuning or {"bin_row_items": 8, "bin_tile_items": 16}
    tx, ty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE
    chunks1 = (n + 64 * tu["bin_row_items"] - 1) // (64 * tu["bin_row_items"])
    chunks2 = R // (64 * tu["bin_tile_items"]) + ty
    if stage == "project":
        per_in = 12 + attr_bytes(dtype) * (3 + 4 + 1 + 3 * (deg + 1) ** 2)
        per_out = 48 + 4 + 4 + 4 + 8
        return n * (per_in + per_out)
    packed = tx <= PACKED_RECT_TILES and ty <= PACKED_RECT_TILES
    if stage == "depth_sort":
        # four 8-bit passes: each reads the keys for its digit counts, then
        # reads keys + values (the first pass makes the values) and writes
        # them (the last pass writes no keys); with the packed rectangles
        # also 8 B of rectangle read in the first pass, then 4 B per pass
        # written and read
        passes = 4 * 4 * n + (4 + 8) * n + (8 + 8) * n * 2 + (8 + 4) * n
        payload = (8 + 4) * n + (4 + 4) * n * 2 + (4 + 4) * n
        return passes + (payload if packed else 0)
    if stage == "bin_row_count":
        # packed rectangles read in depth order, else sorted index read, the
        # rectangle gathered and written in depth order; per (row, chunk) a
        # count written and scanned
        return (n * 4 if packed else n * (4 + 8 + 8)) + ty * chunks1 * (4 + 8)
    if stage == "bin_row_scatter":   # sorted index + rectangle per visible Gaussian, 8-byte row entries out
        return n_vis * (4 + (4 if packed else 8)) + R * 8 + chunks1 * ty * 4
    if stage == "bin_tile_count":    # row entries in; per (chunk, column) count written and scanned; tile offsets
        return R * 8 + chunks2 * tx * (4 + 8) + (tx * ty + 1) * 4
    if stage == "bin_tile_scatter":  # row entries in, chunk prefixes, the values out
        return R * 8 + chunks2 * tx * 4 * 2 + K * 4
    if stage == "blend":             # list entry + 48-byte record per staged entry; rgb, T, n_contrib per pixel
        return stats["staged"] * (4 + 48) + W * H * 20
    raise KeyError(stage)


def cpu_baseline(scene, cam, band_rows: int = 4, band_rows_1t: int = 1, reps: int = 3) -> dict:
    """The FP64 oracle, as it is, on a bounded sample of the same frame, per
    stage, median of ``reps`` runs, with all host cores and with one thread.

    Sample: the whole projection and pair emission of the frame, then the sort,
    tile ranges and compositing of the middle ``band_rows`` tile rows (all
    cores) or ``band_rows_1t`` (one thread).  The frame time extrapolates the
    sort and composite by the band's share of all pairs."""
    import statistics
    import numpy as np
    import oracle
    W, H = cam["width"], cam["height"]
    tx, ty = (W + TILE - 1) // TILE, (H + TILE - 1) // TILE

    def one_run(rows):
        t0 = time.perf_counter()
        proj = oracle.project(scene, cam)
        t1 = time.perf_counter()
        _, keys, values = oracle.bin_pairs(proj)
        t2 = time.perf_counter()
        r0 = ty // 2 - rows // 2
        lo, hi = np.uint64(r0 * tx) << np.uint64(32), np.uint64((r0 + rows) * tx) << np.uint64(32)
        sel = (keys >= lo) & (keys < hi)
        bk, bv = oracle.sort_pairs(keys[sel], values[sel])
        ranges = oracle.tile_ranges(bk, tx * ty)
        t3 = time.perf_counter()
        for tile in range(r0 * tx, (r0 + rows) * tx):
            x0, y0 = (tile % tx) * TILE, (tile // tx) * TILE
            ys, xs = np.mgrid[y0:min(y0 + TILE, H), x0:min(x0 + TILE, W)]
            s, e = ranges[tile]
            oracle.composite_pixels(proj, xs.ravel(), ys.ravel(), bv[s:e])
        t4 = time.perf_counter()
        share = float(sel.sum()) / max(1, len(keys))
        return {"project": t1 - t0, "emit_pairs": t2 - t1, "sort_band": t3 - t2, "composite_band": t4 - t3,
                "share": share}

    out = {}
    cores = oracle.max_threads()
    for label, threads, rows in (("all_cores", 0, band_rows), ("one_thread", 1, band_rows_1t)):
        oracle.set_threads(threads)
        runs = [one_run(rows) for _ in range(reps)]
        med = {k: statistics.median(r[k] for r in runs) for k in runs[0]}
        frame = med["project"] + med["emit_pairs"] + (med["sort_band"] + med["composite_band"]) / max(med["share"],
                                                                                                      1e-9)
        out[label] = {"threads": cores if threads == 0 else 1, "band_tile_rows": rows,
                      "band_pair_share": round(med["share"], 4),
                      "stage_s": {k: round(v, 3) for k, v in med.items() if k != "share"},
                      "frame_s_extrapolated": round(frame, 2), "frames_per_s": 1.0 / frame}
    oracle.set_threads(0)
    allc = out["all_cores"]
    return {"value": allc["frames_per_s"], "unit": "frames/s", "cores": allc["threads"], "kind": "oracle",
            "sample": (f"FP64 oracle, median of {reps} runs per stage: full projection and pair emission of the "
                       f"frame, then sort + composite of the middle {band_rows} tile rows "
                       f"({allc['band_pair_share'] * 100:.1f}% of the pairs) with all {allc['threads']} cores, "
                       f"or of the middle {band_rows_1t} row with one thread; frame time extrapolated by the "
                       f"band's share of the pairs"),
            "per_thread_count": out}


# kernel -> the sources its code comes from (a counter reading stays valid
# while these files are unchanged)
KERNEL_SOURCES = {
    "project_kernel": ["project.hip", "gs_internal.h"],
    "level1_scatter_kernel": ["tile_bin.hip", "gs_internal.h"],
    "level2_scatter_kernel": ["tile_bin.hip", "gs_internal.h"],
    "blend_kernel": ["blend.hip", "blend_stage.h", "gs_internal.h"],
    "blend_queue_kernel": ["blend.hip", "blend_stage.h", "gs_internal.h"],
}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c3.txt")


def stage_kernel(stage: str, dtype: int, deg: int, tuning: dict) -> str:
    """The instantiation a single-kernel stage launches for one view, as the
    profiler names it (template arguments follow the storage dtype, the SH
    degree and the launch shapes)."""
    if stage == "project":
        return f"project_kernel<{dtype}, {deg}, true>"
    if stage == "bin_row_scatter":
        return f"level1_scatter_kernel<{tuning['bin_row_items']}>"
    if stage == "bin_tile_scatter":
        return f"level2_scatter_kernel<{tuning['bin_tile_items']}>"
    if stage == "blend":
        if tuning["blend_tile_group"] < 0:   # the persistent grid over the work queue
            return f"blend_queue_kernel<{tuning['blend_batch']}>"
        return f"blend_kernel<false, {tuning['blend_batch']}>"
    raise KeyError(stage)


def source_digest(kernel: str) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel.split("<")[0]]:
        with open(os.path.join(ROOT, "paper_2607_15951_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def library_digest() -> str:
    """Digest of every library source: a frame's counter reading stays valid
    while none of them changes."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2607_15951_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(os.path.basename(f).encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_frame_traffic(workload: str, variant: str):
    """(fetch, write) HBM bytes per frame over all kernels from the committed
    counter summary, with the launch shapes they were taken with, or None
    when there is none or a library source changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            parts = line.split()
            # frame <workload> <variant> <library digest> <fetch bytes> <write bytes> <tuning>
            if len(parts) >= 7 and parts[0] == "frame" and parts[1] == workload and parts[2] == variant:
                if parts[3] != library_digest():
                    return None
                return {"fetch": float(parts[4]), "write": float(parts[5]), "tuning": parts[6]}
    return None


def read_traffic(kernel: str, workload: str, variant: str):
    """HBM bytes per launch of ``kernel`` from the committed counter summary,
    or None when there is none or the kernel's sources changed since."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 6 and parts[0] == "kernel":
                # kernel <name> <workload> <variant> <digest> <fetch_bytes> <write_bytes>; the name
                # keeps its template arguments with the spaces taken out
                rec[(parts[1], parts[2], parts[3])] = (parts[4], float(parts[5]), float(parts[6]))
    kernel = kernel.replace(" ", "")
    r = rec.get((kernel, workload, variant))
    if r is None or r[0] != source_digest(kernel):
        return None
    return r[1] + r[2]


def kernel_short_name(name: str, templates: bool = True) -> str:
    """'void gsmi::(anonymous namespace)::blend_kernel<false>(gsmi::BlendArgs, ...)'
    -> 'blend_kernel<false>' (or 'blend_kernel' without template arguments)."""
    name = name.replace("(anonymous namespace)::", "")
    name = name.split("(")[0].strip()
    if name.startswith("void "):
        name = name[5:]
    name = name.split("::")[-1] if "<" not in name else name[name.rfind("::", 0, name.index("<")) + 2:]
    return name if templates else name.split("<")[0]


def _csv_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def summarize_stats(path: str) -> str:
    """Markdown table of a rocprofv3 --stats kernel summary (run_kernel_stats.csv)."""
    rows = sorted(_csv_rows(path), key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | avg (us) | min (us) | max (us) | total (ms) | share |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {kernel_short_name(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.3f} | {float(r['Percentage']):.1f}% |")
    return "\n".join(out)


def _pmc_avg(path: str, counter: str) -> dict:
    """Average per dispatch of one counter, by kernel name."""
    acc = {}
    for r in _csv_rows(path):
        # the work-counting blend variant (one launch per bench run) is not the timed kernel
        if r["Counter_Name"] != counter or "blend_kernel<true" in kernel_short_name(r["Kernel_Name"]):
            continue
        k = kernel_short_name(r["Kernel_Name"]).replace(" ", "")
        acc.setdefault(k, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def summarize_pmc(fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str, workload: str,
                  variant: str, tuning: str | None = None) -> str:
    """HBM bytes per launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch),
    each scaled by the reading of a plain copy of known size."""
    copy_bytes = COPY_CALIBRATION_BYTES
    cf = max(_pmc_avg(copy_fetch_csv, "FETCH_SIZE").items(), key=lambda kv: kv[1])
    cw = max(_pmc_avg(copy_write_csv, "WRITE_SIZE").items(), key=lambda kv: kv[1])
    f_fac = copy_bytes / (cf[1] * 1024.0)
    w_fac = copy_bytes / (cw[1] * 1024.0)
    fetch = _pmc_avg(fetch_csv, "FETCH_SIZE")
    write = _pmc_avg(write_csv, "WRITE_SIZE")
    lines = [f"# copy calibration: {cf[0]} FETCH_SIZE {cf[1]:.0f} KiB, WRITE_SIZE {cw[1]:.0f} KiB for "
             f"{copy_bytes} B read and written -> factors fetch {f_fac:.3f}, write {w_fac:.3f}",
             "# kernel <name> <workload> <variant> <source digest> <fetch bytes/launch> <write bytes/launch>"]
    for k in sorted(set(fetch) & set(write)):
        if k.split("<")[0] in KERNEL_SOURCES:
            lines.append(f"kernel {k} {workload} {variant} {source_digest(k)} {fetch[k] * 1024 * f_fac:.0f} "
                         f"{write[k] * 1024 * w_fac:.0f}")
    for k in sorted(set(fetch) | set(write)):
        lines.append(f"# raw {k}: FETCH_SIZE {fetch.get(k, float('nan')):.0f} KiB, "
                     f"WRITE_SIZE {write.get(k, float('nan')):.0f} KiB per dispatch")
    if tuning:
        # a --frames-only run renders whole frames and nothing else: every
        # dispatch belongs to one, and the projection runs once per frame
        ff = _pmc_total(fetch_csv, "FETCH_SIZE")
        ww = _pmc_total(write_csv, "WRITE_SIZE")
        frames = ff["frames"]
        lines.append(f"# frame totals over {frames} frames (every dispatch of a --frames-only run), "
                     "bytes per frame: frame <workload> <variant> <library digest> <fetch> <write> <tuning>")
        lines.append(f"frame {workload} {variant} {library_digest()} {ff['kib'] * 1024 * f_fac / frames:.0f} "
                     f"{ww['kib'] * 1024 * w_fac / frames:.0f} {tuning}")
    return "\n".join(lines)


def _pmc_total(path: str, counter: str) -> dict:
    """Sum of one counter over every dispatch of a run, and the number of
    frames (projection dispatches) it covers."""
    kib, frames = 0.0, 0
    seen = set()
    for r in _csv_rows(path):
        if r["Counter_Name"] != counter:
            continue
        name = kernel_short_name(r["Kernel_Name"], templates=False)
        if name.startswith("__amd_rocclr"):   # the runtime's copies: the scene upload and the size readback
            continue
        kib += float(r["Counter_Value"])
        key = r.get("Dispatch_Id") or r.get("Correlation_Id") or id(r)
        if name == "project_kernel" and key not in seen:
            seen.add(key)
            frames += 1
    return {"kib": kib, "frames": max(frames, 1)}


# the plain copy that calibrates the byte counters: 4 GiB read and written,
# far past the 256 MB last-level cache
COPY_CALIBRATION_BYTES = 1 << 32


def copy_calibration(nbytes: int = COPY_CALIBRATION_BYTES, reps: int = 3):
    """A plain device-to-device copy of known size: reads and writes nbytes
    per launch.  Profiled with the same FETCH_SIZE / WRITE_SIZE counters, it
    gives the factor between counter readings and bytes moved."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_launch": nbytes, "launches": reps}), flush=True)


def time_batched(r, dev, cams, steps: int, autotune: bool = True) -> dict:
    """Views/s of one gs_render_batched call over ``cams`` per step, of the
    same batch replayed as a captured graph, and of the same views rendered by
    one gs_render call each (launch shapes autotuned for the batch first)."""
    import torch
    tuning = r.autotune(dev, cams, reps=3)["tuning"] if autotune else r.tuning()
    outs = r.render_batched(dev, cams)
    torch.cuda.synchronize()
    bsteps = max(3, min(steps, 10))
    t0 = time.perf_counter()
    for _ in range(bsteps):
        r.render_batched(dev, cams, outs=outs)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / bsteps
    info = r.list_info()
    for c, o in zip(cams, outs):   # warm the single-view sizes
        r.render(dev, c, c["width"], c["height"], out=o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(bsteps):
        for c, o in zip(cams, outs):
            r.render(dev, c, c["width"], c["height"], out=o)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3 / bsteps
    # the same batch captured once into a graph (pair capacity 25% above this
    # frame's K) and replayed
    gr = r.graph(dev, cams, pair_capacity=int(info["num_pairs"] * 1.25) + 1024, outs=outs)
    gr.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(bsteps):
        gr.launch()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / bsteps
    gr.close()
    pixels = sum(c["width"] * c["height"] for c in cams)
    return {"views": len(cams), "megapixels": round(pixels / 1e6, 2), "pairs": info["num_pairs"],
            "ms_per_batch": round(ms_batch, 3), "views_per_s": round(len(cams) * 1e3 / ms_batch, 1),
            "ms_per_batch_graph": round(ms_graph, 3), "views_per_s_graph": round(len(cams) * 1e3 / ms_graph, 1),
            "ms_one_call_per_view": round(ms_single, 3),
            "views_per_s_one_call_per_view": round(len(cams) * 1e3 / ms_single, 1), "steps": bsteps,
            "tuning": tuning}


def time_backward(r, dev, cam, W: int, H: int, steps: int, out) -> dict:
    """Device time of gs_render_backward for the frame (seeded dL/d(image) and
    dL/d(final_T) in [0, 1)), alone and after its render (one training
    step's rasterizer work)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(1234)
    gi = torch.rand((3, H, W), device="cuda", generator=g)
    gt = torch.rand((H, W), device="cuda", generator=g)
    r.render(dev, cam, W, H, out=out)
    r.backward(dev, [gi], [gt])
    torch.cuda.synchronize()
    bsteps = max(3, min(steps, 20))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(bsteps):
        r.backward(dev, [gi], [gt])
    e1.record()
    torch.cuda.synchronize()
    ms_bwd = e0.elapsed_time(e1) / bsteps
    t0 = time.perf_counter()
    for _ in range(bsteps):
        r.render(dev, cam, W, H, out=out)
        r.backward(dev, [gi], [gt])
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / bsteps
    return {"ms_backward": round(ms_bwd, 4), "ms_forward_backward": round(ms_step, 4),
            "forward_backward_per_s": round(1e3 / ms_step, 1), "steps": bsteps}


def time_capacity(r, dev, cam, W: int, H: int, steps: int, out, K: int) -> dict:
    """The same frame without the host read of its sizes: with a pair
    capacity of 1.1 K every size is a device-side bound and nothing inside
    the frame waits for the host; as back-to-back gs_render calls, and as
    replays of a captured graph of the render."""
    import torch
    cap = int(K * 1.1)
    bsteps = max(3, min(steps, 50))
    for _ in range(3):
        r.render(dev, cam, W, H, out=out, pair_capacity=cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(bsteps):
        r.render(dev, cam, W, H, out=out, pair_capacity=cap)
    torch.cuda.synchronize()
    ms_cap = (time.perf_counter() - t0) * 1e3 / bsteps
    g = r.graph(dev, [cam], pair_capacity=cap, outs=[out])
    for _ in range(3):
        g.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(bsteps):
        g.launch()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / bsteps
    g.close()
    return {"pair_capacity": cap, "ms_per_step": round(ms_cap, 4), "frames_per_s": round(1e3 / ms_cap, 2),
            "ms_per_step_graph": round(ms_graph, 4), "frames_per_s_graph": round(1e3 / ms_graph, 2),
            "steps": bsteps}


@functools.lru_cache(maxsize=1)
def _workload_scene(workload: str):
    import scenes
    return scenes.make_scene(workload)


def time_workload(r, workload: str, dtype: int, steps: int, graph: bool = False) -> dict:
    """Frame time of another workload's default view (launch shapes as
    autotuned for the main frame), back-to-back gs_render calls, and with
    ``graph`` as replays of a captured graph of the frame."""
    import torch
    import paper_2607_15951_amd as gs
    import scenes
    sc = _workload_scene(workload)
    cam = scenes.make_cameras(workload)[0]
    W, H = cam["width"], cam["height"]
    dev = gs.scene_to_device(sc, dtype)
    out = r.render(dev, cam, W, H)
    for _ in range(3):
        r.render(dev, cam, W, H, out=out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        r.render(dev, cam, W, H, out=out)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    info = r.list_info()
    res = {"workload": scenes.WORKLOAD_NAMES[workload], "attributes": {gs.GS_F32: "fp32", gs.GS_BF16: "bf16",
                                                                       gs.GS_F16: "fp16"}[dtype],
           "width": W, "height": H, "pairs": info["num_pairs"], "us_per_frame": round(ms * 1e3, 1),
           "frames_per_s": round(1e3 / ms, 2), "steps": steps}
    if graph:
        # the frame's launches captured once and replayed (pair capacity 25%
        # above this frame's K): no host read, one launch per frame
        g = r.graph(dev, [cam], pair_capacity=int(info["num_pairs"] * 1.25) + 1024, outs=[out])
        for _ in range(3):
            g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            g.launch()
        torch.cuda.synchronize()
        gms = (time.perf_counter() - t0) * 1e3 / steps
        g.close()
        res.update(us_per_frame_graph=round(gms * 1e3, 1), frames_per_s_graph=round(1e3 / gms, 2))
    del dev, out
    return res


def time_two_streams(dev, cam, W: int, H: int, steps: int, K: int, tuning: dict) -> dict:
    """Frames of the same scene on two contexts and two streams in turn, so
    that one frame's blend (bound by VALU issue) can overlap the next frame's
    projection and sort (bound by memory): the throughput of a stream of
    frames with two in flight, beside the single-stream frame time.  Pair
    capacity 1.1 K, so that no frame waits for the host."""
    import torch
    import paper_2607_15951_amd as gs
    cap = int(K * 1.1)
    rs = [gs.Renderer(0), gs.Renderer(0)]
    sts = [torch.cuda.Stream(), torch.cuda.Stream()]   # default priority
    outs = []
    for r, st in zip(rs, sts):
        r.set_tuning(**tuning)
        with torch.cuda.stream(st):
            o = r.render(dev, cam, W, H, pair_capacity=cap)
            for _ in range(3):
                r.render(dev, cam, W, H, out=o, pair_capacity=cap)
        outs.append(o)
    torch.cuda.synchronize()
    frames = max(4, steps - steps % 2)
    t0 = time.perf_counter()
    for k in range(frames):
        i = k % 2
        with torch.cuda.stream(sts[i]):
            rs[i].render(dev, cam, W, H, out=outs[i], pair_capacity=cap)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / frames
    for r in rs:
        r.close()
    return {"frames": frames, "ms_per_frame": round(ms, 4), "frames_per_s": round(1e3 / ms, 2),
            "pair_capacity": cap}


def time_batched_backward(r, dev, cams, steps: int) -> dict:
    """One training step's rasterizer work on a batch of views: the batched
    render of all views, then one backward over them (seeded dL/d(image) and
    dL/d(final_T) in [0, 1) per view), per step; and the backward alone."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(4321)
    outs = r.render_batched(dev, cams)
    gi = [torch.rand((3, c["height"], c["width"]), device="cuda", generator=g) for c in cams]
    gt = [torch.rand((c["height"], c["width"]), device="cuda", generator=g) for c in cams]
    r.backward(dev, gi, gt)
    torch.cuda.synchronize()
    bsteps = max(3, min(steps, 10))
    t0 = time.perf_counter()
    for _ in range(bsteps):
        r.render_batched(dev, cams, outs=outs)
        r.backward(dev, gi, gt)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / bsteps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(bsteps):
        r.backward(dev, gi, gt)
    e1.record()
    torch.cuda.synchronize()
    ms_bwd = e0.elapsed_time(e1) / bsteps
    # the same step, render (with a pair capacity 25% above this batch's K)
    # and backward, captured into one graph and replayed: one launch per step
    cap = int(r.list_info()["num_pairs"] * 1.25) + 1024
    o2 = r.render_batched(dev, cams, pair_capacity=cap)
    r.backward(dev, gi, gt)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        r.render_batched(dev, cams, pair_capacity=cap, outs=o2)
        r.backward(dev, gi, gt)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(bsteps):
        graph.replay()
    torch.cuda.synchronize()
    ms_graph = (time.perf_counter() - t0) * 1e3 / bsteps
    del graph
    return {"views": len(cams), "ms_forward_backward": round(ms_step, 3), "ms_backward": round(ms_bwd, 3),
            "views_per_s_forward_backward": round(len(cams) * 1e3 / ms_step, 1),
            "ms_forward_backward_graph": round(ms_graph, 3),
            "views_per_s_forward_backward_graph": round(len(cams) * 1e3 / ms_graph, 1), "steps": bsteps}


def time_reuse(r, dev, W: int, H: int, frames: int = 16) -> dict:
    """Orbits of several step sizes around the scene (the camera motions of
    the paper's churn table): frame time with and without
    GS_RENDER_REUSE_ORDER, the depth-sort stage time with it, how many frames
    kept the previous order, the order's descents, and the churn -- the
    share of Gaussians whose tile rectangle changed since the last frame."""
    import torch
    import scenes
    out = {}
    for step in (0.0, 0.001, 0.01, 0.05, 0.1, 0.5, 2.0):
        cams = [scenes.orbit_camera(step * f, W, H) for f in range(frames + 1)]
        o = r.render(dev, cams[0], W, H)
        timed = {}
        for reuse in (True, False):
            r.render(dev, cams[0], W, H, out=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for c in cams[1:]:
                r.render(dev, c, W, H, out=o, reuse_order=reuse)
            torch.cuda.synchronize()
            timed[reuse] = (time.perf_counter() - t0) * 1e3 / frames
        r.render(dev, cams[0], W, H, out=o)
        prev = r.projection()["rect"].clone()
        r.set_profiling(stages=True)
        sort_ms = kept = desc = 0.0
        moved = 0
        for c in cams[1:]:
            r.render(dev, c, W, H, out=o, reuse_order=True)
            sort_ms += r.stage_times()["depth_sort"]
            rep = r.order_reuse()
            kept += rep["reused"]
            desc += rep["descents"]
            rect = r.projection()["rect"]
            moved += int((rect != prev).any(dim=1).sum())
            prev = rect.clone()
        r.set_profiling(stages=False)
        n = int(prev.shape[0])
        out[f"orbit_{step}deg"] = {
            "ms_per_frame_reuse": round(timed[True], 4), "ms_per_frame_plain": round(timed[False], 4),
            "depth_sort_ms_reuse": round(sort_ms / frames, 4), "frames_reused": int(kept), "frames": frames,
            "descents_per_frame": round(desc / frames, 1), "churn_pct": round(100.0 * moved / (frames * n), 3)}
    return out


def time_list_reuse(r, dev, cam, W: int, H: int, frames: int = 20) -> dict:
    """A static camera over frames whose colours change (the SH coefficients
    alternate between two sets, the geometry stays): frame time with
    GS_RENDER_REUSE_LISTS, which keeps the lists when no depth key or tile
    rectangle changed, against plain renders of the same frames, and how many
    frames kept their lists; the same from a captured graph.  Then one orbit
    step per frame, where the lists cannot hold: the cost of the comparison."""
    import torch
    import scenes
    dev_b = dict(dev)
    dev_b["sh"] = (dev["sh"].float() * 0.9).to(dev["sh"].dtype)
    scenes_ab = [dev, dev_b]
    o = r.render(dev, cam, W, H)
    res = {}
    for reuse in (True, False):
        r.render(dev, cam, W, H, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(frames):
            r.render(scenes_ab[(f + 1) % 2], cam, W, H, out=o, reuse_lists=reuse)
        torch.cuda.synchronize()
        res["ms_per_frame_reuse" if reuse else "ms_per_frame_plain"] = round((time.perf_counter() - t0) * 1e3 / frames,
                                                                            4)
    kept = 0
    r.render(dev, cam, W, H, out=o)
    for f in range(frames):
        r.render(scenes_ab[(f + 1) % 2], cam, W, H, out=o, reuse_lists=True)
        kept += r.list_reuse()["reused"]
    res["frames_kept"] = int(kept)
    res["frames"] = frames
    # the same static camera replayed from a captured graph (pair capacity
    # 1.1 K), with and without the flag: the decision is taken on the device
    cap = int(r.list_info()["num_pairs"] * 1.1)
    for reuse in (True, False):
        gr = r.graph(dev, [cam], pair_capacity=cap, reuse_lists=reuse)
        gr.launch()
        gr.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(frames):
            gr.launch()
        torch.cuda.synchronize()
        res["graph_ms_per_frame_reuse" if reuse else "graph_ms_per_frame_plain"] = round(
            (time.perf_counter() - t0) * 1e3 / frames, 4)
        gr.close()
    cams = [scenes.orbit_camera(0.01 * f, W, H) for f in range(frames + 1)]
    for reuse in (True, False):
        r.render(dev, cams[0], W, H, out=o)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in cams[1:]:
            r.render(dev, c, W, H, out=o, reuse_lists=reuse)
        torch.cuda.synchronize()
        key = "orbit_ms_per_frame_reuse" if reuse else "orbit_ms_per_frame_plain"
        res[key] = round((time.perf_counter() - t0) * 1e3 / frames, 4)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C3")
    ap.add_argument("--variant", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the BF16/FP16 storage variants")
    ap.add_argument("--no-autotune", action="store_true", help="time the default launch shapes")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 4 GiB device copy (reference for the HBM byte counters)")
    ap.add_argument("--tuning", metavar="SORT,ROW,TILE,GROUP[,BATCH]",
                    help="launch shapes to use instead of autotuning (sort_items, bin_row_items, bin_tile_items, "
                         "blend_tile_group, blend_batch)")
    ap.add_argument("--batched", action="store_true",
                    help="with --frames-only: render all cameras of the workload in one gs_render_batched call "
                         "per frame (C4: 64 views)")
    ap.add_argument("--reuse-lists", action="store_true",
                    help="with --frames-only: render with GS_RENDER_REUSE_LISTS (the first frame builds the lists, "
                         "the others keep them)")
    ap.add_argument("--frames-only", type=int, metavar="F",
                    help="render F frames of the workload (after one warm-up frame) and nothing else, for "
                         "per-frame counter totals; prints one JSON line")
    ap.add_argument("--summarize-stats", metavar="KERNEL_STATS_CSV",
                    help="print a rocprofv3 --stats kernel summary as a markdown table, then exit")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="print HBM bytes per launch from rocprofv3 --pmc counter files, then exit")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.summarize_stats:
        print(summarize_stats(args.summarize_stats))
        return
    if args.summarize_pmc:
        print(summarize_pmc(*args.summarize_pmc, workload=args.workload, variant=args.variant,
                            tuning=args.tuning))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this single-GPU build "
              "(the render would shard by camera or by screen tiles)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2607_15951_amd as gs
    import scenes

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dtype = {"fp32": gs.GS_F32, "bf16": gs.GS_BF16, "fp16": gs.GS_F16}[args.variant]
    log(f"[bench] generating {args.workload}")
    scene = scenes.make_scene(args.workload)
    cam = scenes.make_cameras(args.workload)[0]
    W, H = cam["width"], cam["height"]
    n = scene["means"].shape[1]
    deg = scene["sh_degree"]
    dev = gs.scene_to_device(scene, dtype)
    r = gs.Renderer(0)
    out = {"image": torch.empty((3, H, W), dtype=torch.float32, device="cuda"),
           "final_T": torch.empty((H, W), dtype=torch.float32, device="cuda"),
           "n_contrib": torch.empty((H, W), dtype=torch.int32, device="cuda")}
    # launch shapes for this workload (speed only: every shape renders the
    # same bits), chosen before the timed region like the warm-up
    tune = None
    if args.tuning:
        names = ("sort_items", "bin_row_items", "bin_tile_items", "blend_tile_group", "blend_batch")
        r.set_tuning(**dict(zip(names, (int(v) for v in args.tuning.split(",")))))
    elif not args.no_autotune and not args.frames_only:
        log("[bench] autotune")
        tune = r.autotune(dev, [cam], reps=5)
        log("[bench] tuning " + json.dumps(tune["tuning"]))
    main_tuning = r.tuning()   # the shapes of the timed frames (later variants retune)
    if args.frames_only:
        cams_all = scenes.make_cameras(args.workload) if args.batched else None
        outs = r.render_batched(dev, cams_all) if args.batched else None
        for _ in range(args.frames_only + 1):
            if args.batched:
                r.render_batched(dev, cams_all, outs=outs, reuse_lists=args.reuse_lists)
            else:
                r.render(dev, cam, W, H, out=out, reuse_lists=args.reuse_lists)
        torch.cuda.synchronize()
        r.close()
        print(json.dumps({"frames": args.frames_only + 1, "workload": args.workload, "tuning": main_tuning}),
              flush=True)
        return
    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        r.render(dev, cam, W, H, out=out)
    torch.cuda.synchronize()

    # frame rate: plain renders back to back (the library's own host read of
    # the pair count is the only synchronisation inside a frame)
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.render(dev, cam, W, H, out=out)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # per-frame device times (HIP events around each render on the render
    # stream, frames still back to back): median and spread
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record()
    for k in range(args.steps):
        r.render(dev, cam, W, H, out=out)
        evs[k + 1].record()
    torch.cuda.synchronize()
    per_frame = sorted(evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps))
    frame_pct = {f"p{q}": round(per_frame[min(len(per_frame) - 1, int(q / 100 * len(per_frame)))], 4)
                 for q in (10, 50, 90)}
    # per-stage device times: HIP events the library records on its stream
    prof_steps = min(args.steps, 20)
    r.set_profiling(stages=True)
    stage_sum = {k: 0.0 for k in gs.STAGES}
    for _ in range(prof_steps):
        r.render(dev, cam, W, H, out=out)
        for k, v in r.stage_times().items():
            stage_sum[k] += v
    info = r.list_info()
    # one more render with the work-counting blend (not timed)
    r.set_profiling(stages=False, blend_work=True)
    r.render(dev, cam, W, H, out=out)
    stats = r.blend_stats()
    r.set_profiling(stages=False)
    stage_ms = {k: v / prof_steps for k, v in stage_sum.items()}
    log("[bench] stages ms " + json.dumps({k: round(v, 4) for k, v in stage_ms.items()}))

    # storage variants of the same frame: attributes other than means in
    # BF16 / FP16 (the error of each against the FP64 render is reported by
    # the full-size parity tests)
    variants = {}
    if not args.no_variants:
        for name, vd in (("bf16", gs.GS_BF16), ("fp16", gs.GS_F16)):
            if vd == dtype:
                continue
            vdev = gs.scene_to_device(scene, vd)
            for _ in range(3):
                r.render(vdev, cam, W, H, out=out)
            vsteps = min(args.steps, 20)
            torch.cuda.synchronize()
            v0 = time.perf_counter()
            for _ in range(vsteps):
                r.render(vdev, cam, W, H, out=out)
            torch.cuda.synchronize()
            vms = (time.perf_counter() - v0) * 1e3 / vsteps
            r.set_profiling(stages=True)
            r.render(vdev, cam, W, H, out=out)
            vst = r.stage_times()
            r.set_profiling(stages=False)
            pb = algorithmic_bytes("project", n, 0, 0, 0, deg, vd, W, H, {})
            variants[name] = {"frames_per_s": round(1e3 / vms, 2), "ms_per_step": round(vms, 4), "steps": vsteps,
                              "project_ms": round(vst["project"], 4),
                              "project_algorithmic_GBps": round(pb / (vst["project"] * 1e-3) / 1e9, 1)}
            del vdev
            log(f"[bench] variant {name}: " + json.dumps(variants[name]))
        if dtype == gs.GS_F32:
            variants["backward"] = time_backward(r, dev, cam, W, H, args.steps, out)
            log("[bench] variant backward: " + json.dumps(variants["backward"]))
            variants["capacity"] = time_capacity(r, dev, cam, W, H, args.steps, out, info["num_pairs"])
            log("[bench] variant capacity: " + json.dumps(variants["capacity"]))
            variants["two_streams"] = time_two_streams(dev, cam, W, H, args.steps, info["num_pairs"], r.tuning())
            log("[bench] variant two_streams: " + json.dumps(variants["two_streams"]))
            variants["reuse_order"] = time_reuse(r, dev, W, H)
            log("[bench] variant reuse_order: " + json.dumps(variants["reuse_order"]))
            variants["reuse_lists"] = time_list_reuse(r, dev, cam, W, H)
            log("[bench] variant reuse_lists: " + json.dumps(variants["reuse_lists"]))
        # batched: the same frame's scene from 8 cameras on a ring (1080p each),
        # and the 64-camera mixed-resolution workload, each one
        # gs_render_batched call per step, against the same views rendered one
        # gs_render call at a time
        if dtype == gs.GS_F32:
            variants["batched_ring8_1080p"] = time_batched(r, dev, scenes.ring_cameras(8, W, H), args.steps)
            log("[bench] variant batched_ring8_1080p: " + json.dumps(variants["batched_ring8_1080p"]))
            del dev
            sc4 = scenes.make_scene("C4")
            dev4 = gs.scene_to_device(sc4)
            variants["batched_C4_64views"] = time_batched(r, dev4, scenes.make_cameras("C4"), args.steps)
            variants["batched_C4_64views"]["workload"] = scenes.WORKLOAD_NAMES["C4"]
            log("[bench] variant batched_C4_64views: " + json.dumps(variants["batched_C4_64views"]))
            variants["batched_C4_64views_backward"] = time_batched_backward(r, dev4, scenes.make_cameras("C4"),
                                                                            args.steps)
            log("[bench] variant batched_C4_64views_backward: " +
                json.dumps(variants["batched_C4_64views_backward"]))
            del dev4
            # the small and the large workloads: C1 (1k Gaussians, 128x128),
            # bound by launch latency, and C5 (6M Gaussians at 3840x2160) with
            # BF16 / FP16 attribute storage
            variants["small_C1"] = time_workload(r, "C1", gs.GS_F32, steps=100, graph=True)
            log("[bench] variant small_C1: " + json.dumps(variants["small_C1"]))
            for name, vd in (("C5_4k_bf16", gs.GS_BF16), ("C5_4k_fp16", gs.GS_F16)):
                variants[name] = time_workload(r, "C5", vd, steps=10)
                log(f"[bench] variant {name}: " + json.dumps(variants[name]))

    K, n_vis, R = info["num_pairs"], info["n_visible"], info["num_row_entries"]
    tuned = main_tuning
    single = ["project", "bin_row_scatter", "bin_tile_scatter", "blend"]
    dom = max(single, key=lambda k: stage_ms[k])
    if dom == "blend":
        flops = FLOPS_EVAL * stats["evaluations"] + FLOPS_COMPOSITE * stats["composited"]
        achieved = flops / (stage_ms[dom] * 1e-3) / 1e12
        kname = stage_kernel(dom, dtype, deg, tuned)
        roof = {"kernel": kname, "bound": "alu", "achieved": round(achieved, 3),
                "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
                "traffic": read_traffic(kname, args.workload, args.variant), "work": {"evaluations": stats["evaluations"], "composited": stats["composited"],
                                          "flops_per_evaluation": FLOPS_EVAL,
                                          "flops_per_composite": FLOPS_COMPOSITE}}
    else:
        by = algorithmic_bytes(dom, n, n_vis, K, R, deg, dtype, W, H, stats, tuned)
        achieved = by / (stage_ms[dom] * 1e-3) / 1e9
        kname = stage_kernel(dom, dtype, deg, tuned)
        roof = {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": read_traffic(kname, args.workload, args.variant),
                "bytes_per_launch": int(by)}
    stage_gbs = {}
    stage_bytes = {}
    for k in gs.STAGES:
        by = algorithmic_bytes(k, n, n_vis, K, R, deg, dtype, W, H, stats, tuned)
        stage_bytes[k] = by
        stage_gbs[k] = round(by / (stage_ms[k] * 1e-3) / 1e9, 1) if stage_ms[k] > 0 else None
    # the whole frame: every stage's algorithmic bytes over the frame time
    frame_bytes = sum(stage_bytes.values())
    frame_gbs = frame_bytes / (ms_per_step * 1e-3) / 1e9
    ft = read_frame_traffic(args.workload, args.variant)
    frame = {"algorithmic_bytes": int(frame_bytes), "achieved_GBps": round(frame_gbs, 1), "peak_GBps": HBM_PEAK_GBS,
             "frac": round(frame_gbs / HBM_PEAK_GBS, 4),
             "stage_algorithmic_bytes": {k: int(v) for k, v in stage_bytes.items()},
             "counter_bytes": None if ft is None else int(ft["fetch"] + ft["write"]),
             "counter_GBps": None if ft is None else round((ft["fetch"] + ft["write"]) / (ms_per_step * 1e-3) / 1e9, 1),
             "counter_tuning": None if ft is None else ft["tuning"]}
    # blend work: the evaluations Eq. 1 needs (each pixel up to its
    # termination) and the lane evaluations the kernel executed (64 per wave
    # and staged entry it did not skip)
    blend_s = stage_ms["blend"] * 1e-3
    blend_work = {**stats,
                  "tflops": round((FLOPS_EVAL * stats["evaluations"] + FLOPS_COMPOSITE * stats["composited"])
                                  / blend_s / 1e12, 3),
                  "tflops_executed": round((FLOPS_EVAL * stats["lane_evaluations"] + FLOPS_COMPOSITE *
                                            stats["composited"]) / blend_s / 1e12, 3),
                  "peak_tflops_nonpacked": FP32_VECTOR_NONPACKED_TFLOPS}
    blend_work["frac_executed"] = round(blend_work["tflops_executed"] / FP32_VECTOR_NONPACKED_TFLOPS, 4)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (FP64 oracle, bounded sample)")
        cpu = cpu_baseline(scene, cam)

    res = {
        "metric": METRIC,
        "value": round(1e3 / ms_per_step, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == gs.GS_F32 else ("f32 compute, bf16 attributes" if dtype == gs.GS_BF16
                                                     else "f32 compute, f16 attributes"),
        "data": "synthetic",
        "config": {"workload": scenes.WORKLOAD_NAMES[args.workload], "gaussians": n, "width": W, "height": H,
                   "sh_degree": deg, "tile": TILE, "attributes": args.variant, "num_pairs": K,
                   "row_entries": R, "visible": n_vis},
        "frame_ms_events": frame_pct,
        "stages_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stages_algorithmic_GBps": stage_gbs,
        "frame_hbm": frame,
        "blend_work": blend_work,
        "roofline": roof,
        "tuning": tune,
        "variants": variants,
        "cpu_baseline": cpu,
    }
    r.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
