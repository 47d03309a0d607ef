#!/usr/bin/env python3
"""Benchmark: 1920x1080 Universal Perspective views of a 1,000,000-triangle
scene (+ enclosing radius-100 icosphere) on one MI355X.

One step = the whole hot path over one batch: per-triangle setup of the
resident scene (vsr_setup_tris) followed by one vsr_submit of `--views`
1080p views (k in {1, 0.5, 0, -0.5} x yaw/pitch orientations), i.e. map
generation (once per distinct lens: the map is camera-frame), binning and
rasterization of every view.  `value` is views per second over the timed
steps (inputs resident in HBM).  The same batch with a distinct lens per
view (64 maps per step) is reported beside it.

Also reported: the plain per-view form (vsr_build_map -> vsr_bin ->
vsr_raster, one view at a time) and its per-view latency percentiles, the
batched form without the setup, the setup alone, the rasterizer's roofline
(algorithmic lane-ops per covered fragment x covered fragments / measured
kernel time, against the FP32 VALU peak), the aliasing-free variant
(vsr_build_map with VSR_MAP_AA -> vsr_bin -> vsr_aa_raster) per view with its
own VALU roofline, the fragment-data step, and the FP64 CPU oracle timed on
a bounded pixel sample on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
       python bench.py --summarize DIR...   (rocprofv3 CSV output -> text summary)
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_VALU_LANE_OPS = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: non-packed FP32 VALU
PEAK_HBM = 8.0e12
OPS_PER_AA_FRAGMENT = 36                     # 3 edge dots (9) + chord (6) + miter (1) + 4 steps (12) + 3 min + cmp + g.N (3) + div
OPS_PER_WIRE_FRAGMENT = 46                   # 3 sides x (dot 3, |.| step 2, chord 6, cap step 2, min 1) + max/compare
OPS_PER_PARTICLE_FRAGMENT = 28               # chord 6, cap step 2, g.N 3, rcp + mul 2, Y = X x N 6, two dots 6, 2 fma, compare
OPS_PER_FRAGMENT = 20                        # 3 edge dots (9) + min3 + cmp + g.N (3) + rcp + mul + cmp64 + 2 sel
BIN_BYTES_PER_TRI = 64                       # cap (16 B) + three edge normals (48 B), read once
BIN_BYTES_PER_TILE = 36                      # tile cap (32 B) read, list length (4 B) written
CALIB_BYTES = 256 << 20                      # copy-like calibration kernel of the profiled run
PROFILES = os.path.join(ROOT, "profiles")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash() -> str:
    """Hash of the kernel sources: counters taken from other sources are stale."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2003_10558_amd", "csrc")
    for f in sorted(os.listdir(csrc)) + ["../../include/vsr.h"]:
        if f.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE summary, scaled by the calibration kernel; None when the
    summary is missing or was taken on other kernel sources."""
    path = os.path.join(PROFILES, "traffic_1080p_1m.txt")
    if not os.path.exists(path):
        return None
    src, calib, rows = None, None, {}
    for line in open(path):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "source":
            src = f[1]
        elif f[0] == "calib":
            calib = dict(zip(f[2::2], map(float, f[3::2])))
        elif f[0] == "kernel":
            rows[f[1]] = dict(zip(f[2::2], map(float, f[3::2])))
    key = "vsr::" + kernel
    if src != source_hash() or calib is None or key not in rows:
        return None
    r = rows[key]
    fetch = r["fetch_kib"] * 1024 / calib["fetch_factor"]
    write = r["write_kib"] * 1024 / calib["write_factor"]
    return {"bytes": fetch + write, "fetch_bytes": fetch, "write_bytes": write, "source": src,
            "counters": "FETCH_SIZE, WRITE_SIZE per dispatch / calibration factor"}


def summarize(dirs):
    """Reduce rocprofv3 CSV output (kernel_stats and counter_collection
    files under `dirs`) to the text summaries kept under profiles/."""
    import csv
    import glob
    stats, counters = [], {}
    for d in dirs:
        stats += glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                name = row["Kernel_Name"].split("(")[0].replace("void ", "").strip()
                key = (name, row["Counter_Name"])
                # rows of one dispatch add up; a counter taken in several runs
                # (one directory each) keeps one entry per run and dispatch
                disp = (f, row.get("Dispatch_Id", ""))
                counters.setdefault(key, {}).setdefault(disp, 0.0)
                counters[key][disp] += float(row["Counter_Value"])
    print(f"source {source_hash()}")
    for f in stats:
        rows = list(csv.DictReader(open(f)))
        print(f"# {'kernel':60s} {'calls':>6s} {'total_us':>11s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} "
              f"{'pct':>6s}")
        for r in rows:
            name = r["Name"].split("(")[0].replace("void ", "").strip()[:60]
            print(f"stat {name:60s} {int(r['Calls']):6d} {float(r['TotalDurationNs']) / 1e3:11.1f} "
                  f"{float(r['AverageNs']) / 1e3:10.2f} {float(r['MinNs']) / 1e3:10.2f} "
                  f"{float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}")
    if counters:
        names = sorted({k[0] for k in counters})
        cnames = sorted({k[1] for k in counters})
        mean = {k: sum(v.values()) / len(v) for k, v in counters.items()}
        cal = [n for n in names if "neg_kernel" in n]
        if cal and (cal[0], "FETCH_SIZE") in mean and (cal[0], "WRITE_SIZE") in mean:
            ff = max(counters[(cal[0], "FETCH_SIZE")].values()) * 1024 / CALIB_BYTES
            wf = max(counters[(cal[0], "WRITE_SIZE")].values()) * 1024 / CALIB_BYTES
            print(f"calib {cal[0].split('<')[0]} bytes {CALIB_BYTES} fetch_factor {ff:.4f} write_factor {wf:.4f}")
        for n in names:
            if not n.startswith("vsr::"):
                continue
            vals = " ".join(f"{c.lower() if c in ('FETCH_SIZE', 'WRITE_SIZE') else c} {mean[(n, c)]:.6g}"
                            for c in cnames if (n, c) in mean)
            vals = vals.replace("fetch_size", "fetch_kib").replace("write_size", "write_kib")
            nd = max(len({d for _, d in counters[(n, c)]}) for c in cnames if (n, c) in counters)
            if (n, "GRBM_GUI_ACTIVE") in mean:
                # busy fractions: SQ_ACTIVE_INST_VALU counts one quad-cycle
                # per wave64 VALU instruction on its SIMD (4 SIMDs per CU) and
                # SQ_ACTIVE_INST_VALU2 the quad-cycles in which a SIMD issued
                # two, so their difference is the SIMD quad-cycles with VALU
                # issue; SQ_LDS_IDX_ACTIVE counts cycles per CU; the GRBM busy
                # count is summed over the 8 XCDs.  The FMA calibration kernel
                # reads valu_busy 0.89 at 89% of the lane peak.
                cu_cycles = 256 * mean[(n, "GRBM_GUI_ACTIVE")] / 8
                if (n, "SQ_ACTIVE_INST_VALU") in mean:
                    v2 = mean.get((n, "SQ_ACTIVE_INST_VALU2"), 0.0)
                    vals += f" valu_busy {(mean[(n, 'SQ_ACTIVE_INST_VALU')] - v2) / cu_cycles:.3f}"
                    if (n, "SQ_ACTIVE_INST_VALU2") in mean:
                        vals += f" valu_dual_frac {v2 / max(1.0, mean[(n, 'SQ_ACTIVE_INST_VALU')]):.3f}"
                if (n, "SQ_LDS_IDX_ACTIVE") in mean:
                    vals += f" lds_busy {mean[(n, 'SQ_LDS_IDX_ACTIVE')] / cu_cycles:.3f}"
            print(f"kernel {n.replace(' ', '')} dispatches {nd} {vals}")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize":
        summarize(sys.argv[2:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--views", type=int, default=64)
    ap.add_argument("--bin-depth", type=int, default=256)
    ap.add_argument("--fmt", choices=["f32", "oct16"], default="f32")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile", action="store_true", help="short run for rocprofv3: no CPU leg, fewer passes")
    ap.add_argument("--no-tune", action="store_true",
                    help="headline batch with 16x16 bin tiles at depth 512 (the autotuner's usual pick on this "
                         "workload) without timing the candidates")
    ap.add_argument("--serve-seconds", type=float, default=60.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-burst-seconds", type=float, default=3.0,
                    help="after the serving run, the same server at 2x the rate for this long (0: skip)")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); a multi-GPU split of this "
              f"workload is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2003_10558_amd import pipeline, vsr

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    fmt = vsr.VSR_MAP_F32 if args.fmt == "f32" else vsr.VSR_MAP_OCT16
    depth = args.bin_depth

    if args.profile:
        # copy-like calibration kernel of known size (reads and writes
        # CALIB_BYTES once) for scaling the HBM traffic counters
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # ---------------- measured roofline denominators (the library's own
    # calibration kernels): streaming copy of 1 GiB, FP32 FMA chains
    csrc_t = torch.empty(1 << 28, dtype=torch.float32, device=dev)
    cdst_t = torch.empty_like(csrc_t)
    cb = []
    for rep in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        vsr.vsr_calib_copy(csrc_t, cdst_t)
        e1.record()
        e1.synchronize()
        if rep:
            cb.append(e0.elapsed_time(e1))
    copy_gbps = 2 * csrc_t.numel() * 4 / (float(np.median(cb)) * 1e-3) / 1e9
    del csrc_t, cdst_t
    fma_out = torch.empty(256 * 32 * 64, dtype=torch.float32, device=dev)  # 32 waves per CU
    fma_iters = 4096
    cf = []
    for rep in range(6):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        vsr.vsr_calib_fma(fma_out, fma_iters)
        e1.record()
        e1.synchronize()
        if rep:
            cf.append(e0.elapsed_time(e1))
    fma_rate = fma_out.numel() * 8 * fma_iters / (float(np.median(cf)) * 1e-3) / 1e12
    del fma_out
    calib = {"hbm_GBps": copy_gbps, "hbm_sheet_GBps": PEAK_HBM / 1e9, "hbm_kernel": "k_calib_copy (1 GiB read + "
             "1 GiB written per launch, median of 5)", "valu_T_lane_fma_per_s": fma_rate,
             "valu_sheet_T_lane_ops_per_s": PEAK_VALU_LANE_OPS / 1e12,
             "valu_kernel": "k_calib_fma (524,288 threads x 8 chains x 4096 FMAs, median of 5)"}
    log(f"measured peaks: copy {copy_gbps:.0f} GB/s (sheet {PEAK_HBM / 1e9:.0f}), FP32 FMA {fma_rate:.2f} T lane-ops/s "
        f"(sheet {PEAK_VALU_LANE_OPS / 1e12:.2f})")

    t0 = time.time()
    tris = synth.scene_1m()
    log(f"scene: {tris.shape[1]} triangles generated in {time.time() - t0:.1f}s")
    scene = pipeline.Scene(tris, device=dev)
    torch.cuda.synchronize()

    views = synth.views_1080p_batch(args.views)

    stream = torch.cuda.current_stream()

    def ev():
        return torch.cuda.Event(enable_timing=True)

    # ---------------- plain per-view path (resident setup)
    frame = pipeline.render(scene, views[0], fmt=fmt, bin_depth=depth)
    torch.cuda.synchronize()
    n_plain = len(views) if not args.profile else 8
    lat, rast, binl, entries = [], [], [], []
    ntiles = ((views[0].width + 7) // 8) * ((views[0].height + 7) // 8)
    for rep in range(2):
        for v in views[:n_plain]:
            e0, ea, e1, e2 = ev(), ev(), ev(), ev()
            e0.record(stream)
            frame.view_eff = vsr.vsr_build_map(v, fmt, 0, frame.map)
            ea.record(stream)
            vsr.vsr_bin(v, fmt, frame.map, scene.setup, scene.ntri, depth, 0, frame.bins)
            e1.record(stream)
            vsr.vsr_raster(v, fmt, frame.map, scene.setup, scene.ntri, frame.bins, depth, frame.tri_id, frame.depth)
            e2.record(stream)
            e2.synchronize()
            if rep == 1:
                lat.append(e0.elapsed_time(e2))
                binl.append(ea.elapsed_time(e1))
                rast.append(e1.elapsed_time(e2))
                # bin list entries written (per-tile counts follow the 256-byte header)
                entries.append(int(frame.bins[256:256 + 4 * ntiles].view(torch.int32).sum().item()))
    overflow = vsr.vsr_bin_overflow(frame.bins)
    lat = np.array(lat)
    plain_ms = float(lat.mean())
    log(f"plain: {plain_ms:.3f} ms/view (p50 {np.percentile(lat, 50):.3f}, p99 {np.percentile(lat, 99):.3f}), "
        f"bin {np.mean(binl):.3f} ms, raster {np.mean(rast):.3f} ms, list entries {np.mean(entries):.0f}, "
        f"overflowed tiles {overflow}")

    # ---------------- fragment data (section 1.1.4) of the last plain frame
    vattr = torch.from_numpy(synth.vertex_attributes(tris.shape[1], 21)).to(dev)
    bary_t = torch.empty((3, views[0].height, views[0].width), dtype=torch.float32, device=dev)
    attr_t = torch.empty((5, views[0].height, views[0].width), dtype=torch.float32, device=dev)
    # the packed copy of vertices and data is made once per scene and data set
    packed = torch.empty(vsr.vsr_resolve_pack_bytes(scene.ntri, 5), dtype=torch.uint8, device=dev)
    pl = []
    for rep in range(3):
        e0, e1 = ev(), ev()
        e0.record(stream)
        vsr.vsr_resolve_pack(scene.xyz, vattr, scene.ntri, 5, packed)
        e1.record(stream)
        e1.synchronize()
        if rep:
            pl.append(e0.elapsed_time(e1))
    pack_ms = float(np.mean(pl))
    rl, gl = [], []
    for rep in range(4):
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        vsr.vsr_resolve_packed(v, fmt, frame.map, packed, scene.ntri, 5, frame.tri_id,
                               vsr.VSR_RESOLVE_NORMALIZE3, bary_t, attr_t)
        e1.record(stream)
        vsr.vsr_resolve(v, fmt, frame.map, scene.xyz, scene.ntri, frame.tri_id, vattr, 5,
                        vsr.VSR_RESOLVE_NORMALIZE3, bary_t, attr_t)
        e2.record(stream)
        e2.synchronize()
        if rep:
            rl.append(e0.elapsed_time(e1))
            gl.append(e1.elapsed_time(e2))
    resolve_ms, resolve_gather_ms = float(np.mean(rl)), float(np.mean(gl))
    del packed
    ids_now = frame.tri_id.reshape(-1)
    winners = int(torch.unique(ids_now[ids_now != -1]).numel())
    P_r = views[0].width * views[0].height
    resolve_bytes = P_r * ((12 if fmt == vsr.VSR_MAP_F32 else 4) + 4 + 4 * (3 + 5)) + winners * (36 + 3 * 5 * 4)
    log(f"resolve (barycentrics + 5 interpolated components): packed {resolve_ms:.3f} ms "
        f"({resolve_bytes / resolve_ms / 1e6:.0f} GB/s algorithmic), from the arrays {resolve_gather_ms:.3f} ms, "
        f"packing once per scene {pack_ms:.3f} ms; {winners} distinct winners")
    del bary_t, attr_t

    # ---------------- aliasing-free coverage (sections 1.1.1, 1.1.2, 1.4), plain per-view path
    aaf = pipeline.render_aa(scene, views[0], fmt=fmt, bin_depth=depth)
    torch.cuda.synchronize()
    n_aa = 16 if not args.profile else 4
    aa_lat, aa_bin, aa_rast, aa_map = [], [], [], []
    for rep in range(2):
        for v in views[:n_aa]:
            e0, ea, e1, e2 = ev(), ev(), ev(), ev()
            e0.record(stream)
            vsr.vsr_build_map(v, fmt, vsr.VSR_MAP_AA, aaf.map)
            ea.record(stream)
            vsr.vsr_bin(v, fmt, aaf.map, scene.setup, scene.ntri, depth, 0, aaf.bins)
            e1.record(stream)
            vsr.vsr_aa_raster(v, fmt, aaf.map, scene.setup, scene.ntri, aaf.bins, depth, aaf.coverage,
                              aaf.depth_pass, aaf.dominant, aaf.lost)
            e2.record(stream)
            e2.synchronize()
            if rep == 1:
                aa_lat.append(e0.elapsed_time(e2))
                aa_map.append(e0.elapsed_time(ea))
                aa_bin.append(ea.elapsed_time(e1))
                aa_rast.append(e1.elapsed_time(e2))
    aa_lost = int(aaf.lost.item())
    aa_ms = float(np.mean(aa_lat))
    aa_stats = torch.zeros(4, dtype=torch.int64, device=dev)
    F_aa, F_aa_proc, aa_tests, aa_skipped = [], [], [], []
    for q in range(4):
        v = views[q]
        pipeline.render_aa(scene, v, fmt=fmt, bin_depth=depth, frame=aaf, stats=aa_stats, no_skip=True)
        torch.cuda.synchronize()
        F_aa.append(int(aa_stats[1].item()))
        pipeline.render_aa(scene, v, fmt=fmt, bin_depth=depth, frame=aaf, stats=aa_stats)
        torch.cuda.synchronize()
        F_aa_proc.append(int(aa_stats[1].item()))
        aa_tests.append(int(aa_stats[0].item()))
        aa_skipped.append(int(aa_stats[2].item()))
    F_aa_mean = float(np.mean(F_aa))
    log(f"aa: {aa_ms:.3f} ms/view (map {np.mean(aa_map):.3f}, bin {np.mean(aa_bin):.3f}, raster "
        f"{np.mean(aa_rast):.3f}), lost pixels {aa_lost}; fragments per frame (all depths) {F_aa}, found with "
        f"skipping {F_aa_proc}, mask evaluations {aa_tests}, triangles skipped {aa_skipped}")

    # ---------------- other map generators (sections 2.2, 2.3), plain per-view path
    lens_views = {
        "equirect_2048x1024": synth.View(2048, 1024, 0, 0, 1, 90, 0, views[1].rot, lens=vsr.VSR_LENS_EQUIRECT),
        "cube_3456x576": synth.View(3456, 576, 0, 0, 1, 90, 0, views[1].rot, lens=vsr.VSR_LENS_CUBE),
        "screens3_1920x1080": synth.View(1920, 1080, 0, 0, 1, 90, 0, views[1].rot, lens=vsr.VSR_LENS_SCREENS,
                                         lens_n=3, lens_p=(60.0,)),
        "vr_1920x1080": synth.View(1920, 1080, 0, 0, 1, 90, 0, views[1].rot, lens=vsr.VSR_LENS_VR,
                                   lens_p=(100.0, 0.42, 0.22, 0.05)),
        "panorama_1920x1080": synth.View(1920, 1080, 0, 0, 1, 90, 0, views[1].rot, lens=vsr.VSR_LENS_PANORAMA,
                                         lens_p=(270.0,)),
        "distorted_k0.5_1920x1080": synth.View(1920, 1080, 0.5, 0.5, 1.0, 180.0, 0, views[1].rot,
                                               lens_p=(0.12, -0.03, 0.01, -0.01, 0.005, -0.005)),
    }
    lens_stats = {}
    for name, lv in lens_views.items():
        lf = pipeline.render(scene, lv, fmt=fmt, bin_depth=depth)
        torch.cuda.synchronize()
        tm, tb, tr = [], [], []
        for rep in range(3 if not args.profile else 2):
            e0, ea, e1, e2 = ev(), ev(), ev(), ev()
            e0.record(stream)
            pipeline.build_map(lv, fmt, 0, lf.map)
            ea.record(stream)
            vsr.vsr_bin(lv, fmt, lf.map, scene.setup, scene.ntri, depth, 0, lf.bins)
            e1.record(stream)
            vsr.vsr_raster(lv, fmt, lf.map, scene.setup, scene.ntri, lf.bins, depth, lf.tri_id, lf.depth)
            e2.record(stream)
            e2.synchronize()
            if rep:
                tm.append(e0.elapsed_time(ea))
                tb.append(ea.elapsed_time(e1))
                tr.append(e1.elapsed_time(e2))
        npx = lv.width * lv.height
        lens_stats[name] = {"map_ms": float(np.mean(tm)), "bin_ms": float(np.mean(tb)), "raster_ms": float(np.mean(tr)),
                            "fps": 1e3 / (np.mean(tm) + np.mean(tb) + np.mean(tr)), "pixels": npx,
                            "overflowed_tiles": vsr.vsr_bin_overflow(lf.bins)}
        log(f"lens {name}: map {np.mean(tm):.3f} ms, bin {np.mean(tb):.3f} ms, raster {np.mean(tr):.3f} ms "
            f"-> {lens_stats[name]['fps']:.0f} frames/s")
        del lf

    # ---------------- wire frame (section 1.2) of the scene's triangle sides
    wv = views[1]
    wf = pipeline.render_wireframe(scene, wv, fmt=fmt, bin_depth=depth)
    torch.cuda.synchronize()
    w_map, w_bin, w_rast = [], [], []
    for rep in range(3 if not args.profile else 2):
        e0, ea, e1, e2 = ev(), ev(), ev(), ev()
        e0.record(stream)
        pipeline.build_map(wv, fmt, vsr.VSR_MAP_AA_LINES, wf.map)
        ea.record(stream)
        vsr.vsr_bin(wv, fmt, wf.map, scene.setup, scene.ntri, depth, 0, wf.bins)
        e1.record(stream)
        vsr.vsr_aa_wireframe(wv, fmt, wf.map, scene.setup, scene.wire_caps(), scene.ntri, wf.bins, depth,
                             wf.coverage, wf.dominant)
        e2.record(stream)
        e2.synchronize()
        if rep:
            w_map.append(e0.elapsed_time(ea))
            w_bin.append(ea.elapsed_time(e1))
            w_rast.append(e1.elapsed_time(e2))
    wstats = torch.zeros(4, dtype=torch.int64, device=dev)
    pipeline.render_wireframe(scene, wv, fmt=fmt, bin_depth=depth, frame=wf, stats=wstats)
    torch.cuda.synchronize()
    wire_evals, wire_frags = int(wstats[0].item()), int(wstats[1].item())
    t_w = float(np.mean(w_rast)) * 1e-3
    roofline_wire = {"bound": "alu", "achieved": OPS_PER_WIRE_FRAGMENT * wire_frags / t_w / 1e12,
                     "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                     "frac": OPS_PER_WIRE_FRAGMENT * wire_frags / t_w / PEAK_VALU_LANE_OPS,
                     "traffic": traffic_from_profiles("k_wire<false>"), "kernel": "k_wire", "kernel_ms": t_w * 1e3,
                     "fragments_per_launch": wire_frags, "ops_per_fragment": OPS_PER_WIRE_FRAGMENT,
                     "mask_evaluations": wire_evals}
    log(f"wire frame 1080p x 1M: map {np.mean(w_map):.3f} ms, bin {np.mean(w_bin):.3f} ms, raster "
        f"{np.mean(w_rast):.3f} ms; {wire_frags} (pixel, triangle) pairs drawn, {wire_evals} evaluated; "
        f"{roofline_wire['achieved']:.2f} T lane-ops/s ({roofline_wire['frac']:.3f} of VALU)")
    del wf

    # ---------------- particles (section 1.3): 10^6 spheres of the small-triangle angular size
    t0 = time.time()
    pscene = pipeline.ParticleScene(synth.particles_1m(), device=dev)
    torch.cuda.synchronize()
    log(f"particles: 10^6 generated and set up in {time.time() - t0:.1f}s")
    pf = pipeline.render_particles(pscene, wv, fmt=fmt, bin_depth=depth)
    torch.cuda.synchronize()
    p_setup, p_map, p_bin, p_rast = [], [], [], []
    for rep in range(3 if not args.profile else 2):
        es, e0, ea, e1, e2 = ev(), ev(), ev(), ev(), ev()
        es.record(stream)
        pscene.refresh()
        e0.record(stream)
        pipeline.build_map(wv, fmt, vsr.VSR_MAP_AA, pf.map)
        ea.record(stream)
        vsr.vsr_bin(wv, fmt, pf.map, pscene.setup, pscene.n, depth, 0, pf.bins)
        e1.record(stream)
        vsr.vsr_aa_particles(wv, fmt, pf.map, pscene.setup, pscene.n, pf.bins, depth, pf.coverage, pf.depth_pass,
                             pf.uv, pf.dominant, pf.lost)
        e2.record(stream)
        e2.synchronize()
        if rep:
            p_setup.append(es.elapsed_time(e0))
            p_map.append(e0.elapsed_time(ea))
            p_bin.append(ea.elapsed_time(e1))
            p_rast.append(e1.elapsed_time(e2))
    pstats = torch.zeros(4, dtype=torch.int64, device=dev)
    pipeline.render_particles(pscene, wv, fmt=fmt, bin_depth=depth, frame=pf, stats=pstats, no_skip=True)
    torch.cuda.synchronize()
    part_frags = int(pstats[1].item())
    pipeline.render_particles(pscene, wv, fmt=fmt, bin_depth=depth, frame=pf, stats=pstats)
    torch.cuda.synchronize()
    part_found, part_evals = int(pstats[1].item()), int(pstats[0].item())
    part_lost = int(pf.lost.item())
    t_p = float(np.mean(p_rast)) * 1e-3
    roofline_particles = {"bound": "alu", "achieved": OPS_PER_PARTICLE_FRAGMENT * part_frags / t_p / 1e12,
                          "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                          "frac": OPS_PER_PARTICLE_FRAGMENT * part_frags / t_p / PEAK_VALU_LANE_OPS,
                          "traffic": traffic_from_profiles("k_aa_raster<false,1>"), "kernel": "k_aa_raster (particles)",
                          "kernel_ms": t_p * 1e3, "fragments_per_launch": part_frags,
                          "ops_per_fragment": OPS_PER_PARTICLE_FRAGMENT}
    log(f"particles 1080p x 10^6: setup {np.mean(p_setup):.3f} ms, map {np.mean(p_map):.3f} ms, bin "
        f"{np.mean(p_bin):.3f} ms, raster {np.mean(p_rast):.3f} ms; fragments {part_frags} (all depths), "
        f"{part_found} found with skipping, {part_evals} evaluated, lost pixels {part_lost}; "
        f"{roofline_particles['achieved']:.2f} T lane-ops/s ({roofline_particles['frac']:.3f} of VALU)")
    del pf, pscene

    # ---------------- single-view fused path (vsr_build_map + vsr_render)
    ffr = pipeline.render_fused(scene, views[0], fmt=fmt)
    torch.cuda.synchronize()
    fl = []
    for v in views[:n_plain]:
        e0, e1 = ev(), ev()
        e0.record(stream)
        pipeline.render_fused(scene, v, fmt=fmt, frame=ffr)
        e1.record(stream)
        e1.synchronize()
        fl.append(e0.elapsed_time(e1))
    fused_ms = float(np.mean(fl))
    log(f"fused single view: {fused_ms:.3f} ms/view")

    # ---------------- fragment counts (instrumented raster, one view per k)
    stats = torch.zeros(4, dtype=torch.int64, device=dev)
    F_all, F_proc, tests_proc = [], [], []
    for q in range(4):
        v = views[q]
        pipeline.render(scene, v, fmt=fmt, bin_depth=depth, frame=frame)
        vsr.vsr_raster_stats(v, fmt, frame.map, scene.setup, scene.ntri, frame.bins, depth, frame.tri_id,
                             frame.depth, stats, True)
        torch.cuda.synchronize()
        F_all.append(int(stats[1].item()))
        vsr.vsr_raster_stats(v, fmt, frame.map, scene.setup, scene.ntri, frame.bins, depth, frame.tri_id,
                             frame.depth, stats, False)
        torch.cuda.synchronize()
        F_proc.append(int(stats[1].item()))
        tests_proc.append(int(stats[0].item()))
    F_mean = float(np.mean(F_all))
    log(f"covered fragments per frame (k sweep): {F_all}; processed with early exit: {F_proc}; "
        f"tests executed: {tests_proc}")

    # ---------------- batched: setup + one submit of all views per step, in
    # the submit mode, bin tile size and bin depth the autotuner picks for
    # this scene and view size (timed over its candidates before the run)
    from paper_2003_10558_amd import autotune
    tuner = autotune.Tuner(None, reps=3)
    if args.no_tune:
        # what the tuner picks on the benchmark workload
        choice = (vsr.VSR_SUBMIT_BINNED | vsr.VSR_SUBMIT_BIN_TILE16, 512)
        tuner_ms = None
    else:
        choice = tuner.choose(scene, views, fmt)
        tuner_ms = next(iter(tuner.cache.values()))["ms"]
    tuned = autotune.describe(choice)
    log(f"autotuner: {tuned} (candidates, ms per submit: {tuner_ms})")
    batch = pipeline.Batch([(scene, v) for v in views], fmt=fmt, mode=choice[0], bin_depth=choice[1])
    for _ in range(args.warmup):
        scene.refresh()
        batch.submit()
    torch.cuda.synchronize()
    # the library records four events per step between its stages (maps |
    # binner | rasterizer), on the stream its kernels run on
    stage_ev = [[ev() for _ in range(4)] for _ in range(args.steps)]
    for evs in stage_ev:
        for e in evs:
            e.record(stream)  # creates the events before the library records them
    e_start, e_end = ev(), ev()
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e_start.record(stream)
    for k in range(args.steps):
        scene.refresh()
        batch.submit(events=stage_ev[k])
    e_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    step_ms = e_start.elapsed_time(e_end) / args.steps
    views_per_s = len(views) / (step_ms / 1e3)
    stage_map_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in stage_ev]))
    stage_bin_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in stage_ev]))
    stage_raster_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in stage_ev]))
    log(f"batched step, serial (setup + {len(views)} views): {step_ms:.3f} ms -> {views_per_s:.1f} views/s "
        f"(wall {wall:.3f}s for {args.steps} steps); stages: maps {stage_map_ms:.3f} ms, binner "
        f"{stage_bin_ms:.3f} ms, rasterizer {stage_raster_ms:.3f} ms")
    serial = {"ms_per_step": step_ms, "views_per_s": views_per_s, "stage_ms": {
        "maps": stage_map_ms, "binner": stage_bin_ms, "rasterizer": stage_raster_ms}}

    # ---------------- the headline: the same steps pipelined.  Every step
    # still runs its full setup and its submit inside the timed region, but
    # consecutive steps alternate between two streams (two setup buffers of
    # the scene and two batches), so step k+1's setup, and the start of its
    # submit, run beside step k's rendering: the setup's short,
    # latency-bound kernels and the stage boundaries fill the chip.  On each
    # stream a step's submit follows its own setup, and a setup follows the
    # submit that last read its buffer.
    scene_b = pipeline.Scene(scene.xyz, device=dev)
    batch_b = pipeline.Batch([(scene_b, v) for v in views], fmt=fmt, mode=choice[0], bin_depth=choice[1])
    p_scenes, p_batches = [scene, scene_b], [batch, batch_b]
    p_streams = [stream, torch.cuda.Stream(device=dev)]

    def pipelined(nsteps, stage=None, start=None):
        if start is not None:
            p_streams[1].wait_event(start)
        for k in range(nsteps):
            q = k % 2
            p_scenes[q].refresh(p_streams[q])
            p_batches[q].submit(p_streams[q], events=None if stage is None else stage[k])
        joined = torch.cuda.Event()
        joined.record(p_streams[1])
        stream.wait_event(joined)

    p_stage = None
    if args.profile:
        # a profiled run's kernel trace is compared with the serial step's
        # kernel times, so it holds no concurrent steps
        step_ms, views_per_s, pipelined_same = serial["ms_per_step"], serial["views_per_s"], None
        log("profile run: the pipelined leg is skipped")
    else:
        pipelined(max(2, args.warmup))
        torch.cuda.synchronize()
        p_ev = [[ev() for _ in range(4)] for _ in range(args.steps)]
        for evs in p_ev:
            for e in evs:
                e.record(stream)
        e_start, e_end = ev(), ev()
        torch.cuda.synchronize()
        t_wall = time.perf_counter()
        e_start.record(stream)
        pipelined(args.steps, p_ev, e_start)
        e_end.record(stream)  # after both streams' last submits
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_wall
        step_ms = e_start.elapsed_time(e_end) / args.steps
        views_per_s = len(views) / (step_ms / 1e3)
        # stage intervals on each step's stream: they include the other
        # stream's work running beside them, so the kernel rooflines use the
        # serial step's stage times
        p_stage = {"maps": float(np.mean([e[0].elapsed_time(e[1]) for e in p_ev])),
                   "binner": float(np.mean([e[1].elapsed_time(e[2]) for e in p_ev])),
                   "rasterizer": float(np.mean([e[2].elapsed_time(e[3]) for e in p_ev]))}
        pipelined_same = all(torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
                             for a, b in zip(batch.outputs, batch_b.outputs))
        log(f"batched step, steps alternating two streams: {step_ms:.3f} ms -> {views_per_s:.1f} views/s (wall "
            f"{wall:.3f}s for {args.steps} steps); stage intervals (with the other stream's work beside them): "
            f"maps {p_stage['maps']:.3f} ms, binner {p_stage['binner']:.3f} ms, rasterizer "
            f"{p_stage['rasterizer']:.3f} ms; both buffers' images identical: {pipelined_same}")
    del batch_b, scene_b
    # outside the timed region: one view of the batch equals the plain path,
    # bit for bit (ids and depth), at the benchmark's own size and settings
    chk = views[5 % len(views)]
    ref_frame = pipeline.render(scene, chk, fmt=fmt, bin_depth=depth)
    torch.cuda.synchronize()
    b_ids, b_dep = batch.outputs[5 % len(views)]
    batched_equals_plain = bool(torch.equal(b_ids, ref_frame.tri_id) and
                                torch.equal(b_dep.view(torch.int32), ref_frame.depth.view(torch.int32)))
    log(f"batched view {5 % len(views)} == plain render: {batched_equals_plain}")
    del ref_frame

    # batched without setup, and setup alone
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(args.steps):
        batch.submit()
    e1.record(stream)
    torch.cuda.synchronize()
    submit_ms = e0.elapsed_time(e1) / args.steps
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(args.steps):
        scene.refresh()
    e1.record(stream)
    torch.cuda.synchronize()
    setup_ms = e0.elapsed_time(e1) / args.steps
    log(f"submit only: {submit_ms:.3f} ms ({len(views) / submit_ms * 1e3:.1f} views/s); setup {setup_ms:.3f} ms")
    # the same step with every view on its own lens (no map shared)
    dviews = [synth.View(v.width, v.height, v.k + 1e-3 * (q + 1), v.l, v.s, v.omega_deg, v.aov, v.rot)
              for q, v in enumerate(views)]
    dbatch = pipeline.Batch([(scene, v) for v in dviews], fmt=fmt, mode=vsr.VSR_SUBMIT_BINNED, bin_depth=depth)
    dbatch.submit()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(args.steps):
        dbatch.submit()
    e1.record(stream)
    torch.cuda.synchronize()
    dsubmit_ms = e0.elapsed_time(e1) / args.steps
    n_lens = len({(v.width, v.height, v.aov, v.k, v.l, v.s, v.omega_deg) for v in views})
    log(f"submit, {len(views)} distinct lenses: {dsubmit_ms:.3f} ms ({len(views) / dsubmit_ms * 1e3:.1f} views/s); "
        f"the benchmark batch shares {n_lens} lens maps")
    del dbatch
    # the same step with the other bin tile size (8x8 lists, or 16x16 lists
    # culled per 16x8 strip by the rasterizer), at the 8x8 default depth or 512
    other16 = tuned["tile"] == 8
    tbatch = pipeline.Batch([(scene, v) for v in views], fmt=fmt,
                            mode=vsr.VSR_SUBMIT_BINNED | (vsr.VSR_SUBMIT_BIN_TILE16 if other16 else 0),
                            bin_depth=512 if other16 else depth)
    tbatch.submit()
    torch.cuda.synchronize()
    t16_ev = [[ev() for _ in range(4)] for _ in range(args.steps)]
    for evs in t16_ev:
        for e in evs:
            e.record(stream)
    e0, e1 = ev(), ev()
    e0.record(stream)
    for k in range(args.steps):
        scene.refresh()
        tbatch.submit(events=t16_ev[k])
    e1.record(stream)
    torch.cuda.synchronize()
    t16_step_ms = e0.elapsed_time(e1) / args.steps
    t16_bin_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in t16_ev]))
    t16_raster_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in t16_ev]))
    t16_same = all(torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
                   for a, b in zip(tbatch.outputs, batch.outputs))
    log(f"batched step, {16 if other16 else 8}x{16 if other16 else 8} bin tiles: {t16_step_ms:.3f} ms "
        f"({len(views) / t16_step_ms * 1e3:.1f} views/s); "
        f"binner {t16_bin_ms:.3f} ms, rasterizer {t16_raster_ms:.3f} ms; overflowed "
        f"{vsr.vsr_bin_overflow(tbatch.workspace, True)}; images identical to 8x8 bins: {t16_same}")
    del tbatch
    # the tuned step with the persistent rasterizer (work counters) in place
    # of one workgroup per tile group: same images, measured beside it
    pbatch = pipeline.Batch([(scene, v) for v in views], fmt=fmt, mode=choice[0] | vsr.VSR_SUBMIT_PERSISTENT,
                            bin_depth=choice[1])
    pbatch.submit()
    torch.cuda.synchronize()
    p_ev = [[ev() for _ in range(4)] for _ in range(args.steps)]
    for evs in p_ev:
        for e in evs:
            e.record(stream)
    torch.cuda.synchronize()
    for k in range(args.steps):
        pbatch.submit(events=p_ev[k])
    torch.cuda.synchronize()
    p_raster_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in p_ev]))
    p_same = all(torch.equal(a[0], b[0]) and torch.equal(a[1].view(torch.int32), b[1].view(torch.int32))
                 for a, b in zip(pbatch.outputs, batch.outputs))
    grid_raster_ms = serial["stage_ms"]["rasterizer"]
    log(f"persistent rasterizer: {p_raster_ms:.3f} ms against {grid_raster_ms:.3f} ms for the per-tile grid; "
        f"images identical: {p_same}")
    persistent = {"rasterizer_ms": p_raster_ms, "grid_rasterizer_ms": grid_raster_ms, "identical_images": p_same}
    del pbatch
    # the fused depth-sliced batch on the same views
    fbatch = pipeline.Batch([(scene, v) for v in views], fmt=fmt, mode=vsr.VSR_SUBMIT_FUSED)
    fbatch.submit()
    torch.cuda.synchronize()
    e0, e1 = ev(), ev()
    e0.record(stream)
    for _ in range(max(1, args.steps // 2)):
        fbatch.submit()
    e1.record(stream)
    torch.cuda.synchronize()
    fsubmit_ms = e0.elapsed_time(e1) / max(1, args.steps // 2)
    log(f"fused submit: {fsubmit_ms:.3f} ms ({len(views) / fsubmit_ms * 1e3:.1f} views/s)")
    del fbatch

    # ---------------- serving: Poisson arrivals over three resident scenes
    serve_stats = None
    if args.serve_seconds > 0 and not args.profile:
        from paper_2003_10558_amd import serve
        t0 = time.time()
        sc_np = synth.serve_scenes()
        sc = [pipeline.Scene(t, device=dev) for t in sc_np]
        torch.cuda.synchronize()
        log(f"serving scenes {[t.shape[1] for t in sc_np]} ready in {time.time() - t0:.1f}s")
        reqs = serve.make_requests(len(sc), rate_hz=args.serve_rate, duration_s=args.serve_seconds,
                                   seed=synth.SERVE_ARRIVAL_SEED, view_seed=synth.SERVE_ARRIVAL_SEED + 100,
                                   resolutions=synth.SERVE_RESOLUTIONS)
        # the autotuner's (mode, bin tile, depth) per resident scene, timed on
        # 16 request-like views (mixed resolutions) of that scene
        sample_views = synth.random_views(16, 777, resolutions=synth.SERVE_RESOLUTIONS)
        serve_choice = {q: tuner.choose(sc[q], sample_views, fmt) for q in range(len(sc))}
        log(f"serving: autotuned per scene {[autotune.describe(serve_choice[q]) for q in range(len(sc))]}")
        srv = serve.Server(sc, streams=3, max_batch=32, hbm_budget_bytes=int(args.serve_budget_gb * (1 << 30)),
                           mode_for_scene=lambda s: serve_choice[s])
        warm = serve.make_requests(len(sc), rate_hz=200.0, duration_s=0.1, seed=99, view_seed=98,
                                   resolutions=synth.SERVE_RESOLUTIONS)
        srv.run(warm)
        st = srv.run(reqs)
        serve_stats = st.as_dict()
        serve_stats.update({"rate_hz": args.serve_rate, "duration_s": args.serve_seconds,
                            "scenes": [int(t.shape[1]) for t in sc_np],
                            "mode_per_scene": [autotune.describe(serve_choice[q]) for q in range(len(sc))],
                            "resolutions": [list(r) for r in synth.SERVE_RESOLUTIONS]})
        log(f"serving: offered {st.offered} at {args.serve_rate:.0f}/s for {args.serve_seconds}s: completed "
            f"{st.completed}, dropped {st.dropped}, {st.views_per_s:.1f} views/s, p50 {st.p50_ms:.1f} ms, "
            f"p99 {st.p99_ms:.1f} ms, mean batch {st.mean_batch:.1f}, overlapped batches {st.overlapped_batches} of "
            f"{st.batches} (at most {st.max_concurrent_batches} at once); batch sizes {st.batch_size_hist}; "
            f"queue depth at admission {st.queue_depth_hist}; queue wait (ms) {st.queue_wait_hist_ms}")
        # the same server under a burst at 2x the rate: more requests arrive
        # while batches run, so admission forms larger batches
        if args.serve_burst_seconds > 0:
            breqs = serve.make_requests(len(sc), rate_hz=2 * args.serve_rate, duration_s=args.serve_burst_seconds,
                                        seed=synth.SERVE_ARRIVAL_SEED + 1, view_seed=synth.SERVE_ARRIVAL_SEED + 101,
                                        resolutions=synth.SERVE_RESOLUTIONS)
            bt = srv.run(breqs)
            serve_stats["burst"] = {k: v for k, v in bt.as_dict().items()
                                    if k in ("offered", "completed", "dropped", "views_per_s", "p50_ms", "p99_ms",
                                             "queue_p50_ms", "queue_p99_ms", "batches", "mean_batch",
                                             "batch_size_hist", "overlapped_batches", "max_concurrent_batches")}
            serve_stats["burst"].update({"rate_hz": 2 * args.serve_rate, "duration_s": args.serve_burst_seconds})
            log(f"serving burst: offered {bt.offered} at {2 * args.serve_rate:.0f}/s for "
                f"{args.serve_burst_seconds}s: completed {bt.completed}, {bt.views_per_s:.1f} views/s, p50 "
                f"{bt.p50_ms:.1f} ms, p99 {bt.p99_ms:.1f} ms, mean batch {bt.mean_batch:.1f}, batch sizes "
                f"{bt.batch_size_hist}")
        del sc, srv

    # ---------------- rooflines
    P = views[0].width * views[0].height
    map_px = 12 if fmt == vsr.VSR_MAP_F32 else 4
    # bytes per frame with the scene resident: map read, the raw vertices
    # (36 B per triangle) read, ids and depth written
    frame_bytes = map_px * P + 36 * tris.shape[1] + 8 * P
    # dominant kernel of the headline step: the batched binner; its launch
    # covers len(views) frames, timed live between the library's stage
    # events over the timed steps
    nblk_all = len(views) * (((views[0].width + 31) // 32) * ((views[0].height + 31) // 32))
    cap_all = max(64, 1 << (choice[1] - 1).bit_length())
    if tuned["mode"] == "fused":
        sub_bin_kernel = "k_submit_fused"
    elif tuned["tile"] == 16:
        sub_bin_kernel = "k_submit_bin_block16" if (nblk_all >= 2560 and cap_all <= 1024) else "k_submit_bin16"
    else:
        sub_bin_kernel = "k_submit_bin_block" if (nblk_all >= 2560 and cap_all <= 256) else "k_submit_bin"
    t_sb = stage_bin_ms * 1e-3
    roofline_submit_bin = {"bound": "hbm", "achieved": frame_bytes * len(views) / t_sb / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": frame_bytes * len(views) / t_sb / PEAK_HBM,
                "traffic": traffic_from_profiles(sub_bin_kernel), "kernel": sub_bin_kernel,
                "kernel_ms": stage_bin_ms, "frames_per_launch": len(views),
                "algorithmic_bytes": frame_bytes * len(views), "bytes_per_frame": frame_bytes,
                "measured_peak": calib["hbm_GBps"], "frac_of_measured": frame_bytes * len(views) / t_sb / 1e9 /
                calib["hbm_GBps"]}
    # the batched rasterizer against the VALU peak: 20 lane-ops per covered
    # fragment of every frame of the launch
    t_sr = stage_raster_ms * 1e-3
    roofline_submit_raster = {"bound": "alu", "achieved": OPS_PER_FRAGMENT * F_mean * len(views) / t_sr / 1e12,
                              "peak": PEAK_VALU_LANE_OPS / 1e12, "unit": "T lane-ops/s",
                              "frac": OPS_PER_FRAGMENT * F_mean * len(views) / t_sr / PEAK_VALU_LANE_OPS,
                              "kernel": "k_submit_raster16" if tuned["tile"] == 16 else "k_submit_raster",
                              "kernel_ms": stage_raster_ms,
                              "fragments_per_launch": F_mean * len(views), "ops_per_fragment": OPS_PER_FRAGMENT,
                              "measured_peak": calib["valu_T_lane_fma_per_s"],
                              "traffic": traffic_from_profiles("k_submit_raster16" if tuned["tile"] == 16
                                                               else "k_submit_raster")}
    # the headline roofline is the step's dominant kernel: the longer stage
    roofline = dict(roofline_submit_raster if stage_raster_ms >= stage_bin_ms else roofline_submit_bin)
    roofline["dominant_of"] = {"binner_ms": stage_bin_ms, "rasterizer_ms": stage_raster_ms}
    # the plain path's binner (16x16 super-tiles at one 1080p view) with its
    # own HBM ideal: read every triangle's 64-byte bin record and every tile
    # cap once, write the lists
    t_b = float(np.mean(binl)) * 1e-3
    bin_bytes = BIN_BYTES_PER_TRI * tris.shape[1] + BIN_BYTES_PER_TILE * ntiles + 4 * float(np.mean(entries))
    nblk = ((views[0].width + 31) // 32) * ((views[0].height + 31) // 32)
    bin_kernel = "k_bin_block" if (nblk >= 2560 and max(64, 1 << (depth - 1).bit_length()) <= 256) else "k_bin"
    roofline_plain_bin = {"bound": "hbm", "achieved": bin_bytes / t_b / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                          "frac": bin_bytes / t_b / PEAK_HBM, "traffic": traffic_from_profiles(bin_kernel),
                          "kernel": bin_kernel, "kernel_ms": t_b * 1e3, "algorithmic_bytes": bin_bytes,
                          "list_entries": float(np.mean(entries))}
    # the rasterizer against the VALU peak: lane-ops per covered fragment
    t_r = float(np.mean(rast)) * 1e-3
    achieved = OPS_PER_FRAGMENT * F_mean / t_r
    roofline_raster = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                       "unit": "T lane-ops/s", "frac": achieved / PEAK_VALU_LANE_OPS,
                       "traffic": traffic_from_profiles("k_raster<false>"), "kernel": "k_raster",
                       "kernel_ms": t_r * 1e3, "fragments_per_launch": F_mean, "ops_per_fragment": OPS_PER_FRAGMENT}
    # fragment data: HBM-bound (map, ids and outputs per pixel, the winners'
    # vertices and data once each)
    roofline_resolve = {"bound": "hbm", "achieved": resolve_bytes / (resolve_ms * 1e-3) / 1e9,
                        "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                        "frac": resolve_bytes / (resolve_ms * 1e-3) / PEAK_HBM,
                        "traffic": traffic_from_profiles("k_resolve<true>"), "kernel": "k_resolve<true>",
                        "kernel_ms": resolve_ms, "algorithmic_bytes": resolve_bytes, "winners": winners,
                        "unpacked_ms": resolve_gather_ms, "pack_ms": pack_ms}
    # aliasing-free raster against the VALU peak: lane-ops per fragment (all depths)
    t_aa = float(np.mean(aa_rast)) * 1e-3
    achieved_aa = OPS_PER_AA_FRAGMENT * F_aa_mean / t_aa
    roofline_aa = {"bound": "alu", "achieved": achieved_aa / 1e12, "peak": PEAK_VALU_LANE_OPS / 1e12,
                   "unit": "T lane-ops/s", "frac": achieved_aa / PEAK_VALU_LANE_OPS,
                   "traffic": traffic_from_profiles("k_aa_raster<false,0>"), "kernel": "k_aa_raster",
                   "kernel_ms": t_aa * 1e3, "fragments_per_launch": F_aa_mean,
                   "ops_per_fragment": OPS_PER_AA_FRAGMENT}
    # the whole batched step (setup included) per view: covered-fragment
    # work and frame bytes
    per_view_s = step_ms * 1e-3 / len(views)
    roofline_step = {"valu_frac": OPS_PER_FRAGMENT * F_mean / per_view_s / PEAK_VALU_LANE_OPS,
                     "hbm_frac": frame_bytes / per_view_s / PEAK_HBM, "per_view_us": per_view_s * 1e6,
                     "valu_frac_of_measured": OPS_PER_FRAGMENT * F_mean / per_view_s / 1e12 /
                     calib["valu_T_lane_fma_per_s"],
                     "hbm_frac_of_measured": frame_bytes / per_view_s / 1e9 / calib["hbm_GBps"],
                     "per_view_us_stages": {"setup": setup_ms * 1e3 / len(views),
                                            "maps": stage_map_ms * 1e3 / len(views),
                                            "binner": stage_bin_ms * 1e3 / len(views),
                                            "rasterizer": stage_raster_ms * 1e3 / len(views)}}
    log(f"roofline: k_aa_raster {roofline_aa['achieved']:.2f} T lane-ops/s ({roofline_aa['frac']:.3f} of VALU)")
    log(f"roofline (dominant kernel {roofline['kernel']}): {roofline_submit_bin['kernel']} "
        f"{roofline_submit_bin['achieved']:.0f} GB/s ({roofline_submit_bin['frac']:.3f} of HBM, "
        f"{roofline_submit_bin['frac_of_measured']:.3f} of the measured copy rate), {roofline_submit_raster['kernel']} "
        f"{roofline_submit_raster['achieved']:.2f} T lane-ops/s ({roofline_submit_raster['frac']:.3f} of VALU), "
        f"plain k_raster {roofline_raster['frac']:.3f} of VALU, step per view "
        f"{roofline_step['valu_frac']:.3f} VALU / {roofline_step['hbm_frac']:.3f} HBM")

    # ---------------- CPU baseline: the FP64 oracle on a bounded sample
    cpu = None
    if not args.no_cpu and not args.profile:
        import oracle
        oracle.build(force=False)
        v = views[1]
        cores = os.cpu_count() or 1
        # a probe long enough that thread start-up does not inflate the
        # per-pixel time the sample is sized from
        probe = synth.pixel_sample(v.width, v.height, seed=7, n_tiles=0, n_pixels=512)
        t0 = time.perf_counter()
        oracle.render(v, tris, probe, threads=cores)
        t_probe = time.perf_counter() - t0
        n_pix = int(max(64, min(200000, len(probe) * args.cpu_seconds / max(t_probe, 1e-3))))
        sample = synth.pixel_sample(v.width, v.height, seed=8, n_tiles=0, n_pixels=n_pix)
        t0 = time.perf_counter()
        oracle.render(v, tris, sample, threads=cores)
        t_cpu = time.perf_counter() - t0
        tests_per_s = len(sample) * tris.shape[1] / t_cpu
        frames_per_s = tests_per_s / (v.width * v.height * tris.shape[1])
        cpu = {"value": frames_per_s, "unit": "frames/s (extrapolated from a pixel sample)", "cores": cores,
               "kind": "oracle", "sample": f"{len(sample)} random pixels of one 1920x1080 k=0.5 view x "
                                           f"{tris.shape[1]} triangles (brute force), {t_cpu:.1f}s",
               "pixel_triangle_tests_per_s": tests_per_s}
        log(f"cpu oracle: {tests_per_s:.3e} tests/s on {cores} threads -> {frames_per_s:.3e} frames/s")

    out = {
        "metric": "frames/s @1080p·1M tris (batched vs plain); p50/p99 view latency",
        "value": views_per_s,
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fmt == vsr.VSR_MAP_F32 else "f32 (oct16 map)",
        "data": "synthetic",
        "config": {"workload": "1920x1080 Universal Perspective views (k in {1@90deg, 0.5, 0, -0.5 @180deg}, "
                               "l=0.5, s=1, varied yaw/pitch) of 1,000,000 small triangles (angular edge "
                               "~N(0.02,0.005^2) rad, distance U(1,50)) + radius-100 icosphere, seed 1",
                   "views_per_step": len(views), "triangles": int(tris.shape[1]),
                   "submit_mode": tuned["mode"], "bin_tile": tuned["tile"], "bin_depth": tuned["bin_depth"],
                   "chosen_by": "autotuner" if not args.no_tune else "fixed (--no-tune)",
                   "step": "vsr_setup_tris + vsr_submit(all views); consecutive steps alternate between two "
                           "streams, so the next step's setup overlaps this step's rendering"},
        "batched_fps_with_setup": views_per_s,
        "batched_serial": serial,
        "pipelined_buffers_identical": pipelined_same,
        "batched_fps": len(views) / submit_ms * 1e3,
        "batched_fps_distinct_lenses": len(views) / dsubmit_ms * 1e3,
        "lens_maps_per_step": n_lens,
        "plain_fps": 1e3 / plain_ms,
        "plain_view_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "setup_ms": setup_ms,
        "covered_fragments_per_frame": F_mean,
        "processed_fragments_per_frame": float(np.mean(F_proc)),
        "executed_tests_per_frame": float(np.mean(tests_proc)),
        # the same per-frame counts at the batched throughput
        "covered_fragments_per_s": F_mean * views_per_s,
        "executed_tests_per_s": float(np.mean(tests_proc)) * views_per_s,
        "overflowed_tiles_plain": overflow,
        "fused_fps": 1e3 / fused_ms,
        "batched_fused_fps": len(views) / fsubmit_ms * 1e3,
        "batched_persistent": persistent,
        "batched_other_tile": {"tile": 16 if other16 else 8, "fps_with_setup": len(views) / t16_step_ms * 1e3,
                               "binner_ms": t16_bin_ms, "rasterizer_ms": t16_raster_ms,
                               "identical_images": t16_same},
        "autotuned": tuned,
        "autotuner_ms_per_submit": tuner_ms,
        "serving": serve_stats,
        "roofline": roofline,
        "roofline_submit_bin": roofline_submit_bin,
        "roofline_submit_raster": roofline_submit_raster,
        "roofline_plain_bin": roofline_plain_bin,
        "roofline_raster": roofline_raster,
        "measured_peaks": calib,
        "batched_equals_plain": batched_equals_plain,
        "stage_ms": {"maps": stage_map_ms, "binner": stage_bin_ms, "rasterizer": stage_raster_ms},
        "pipelined_stage_intervals_ms": p_stage,
        "roofline_step": roofline_step,
        "roofline_resolve": roofline_resolve,
        "resolve_ms": resolve_ms,
        "aa": {"fps": 1e3 / aa_ms, "ms_per_view": aa_ms, "map_ms": float(np.mean(aa_map)),
               "bin_ms": float(np.mean(aa_bin)), "raster_ms": float(np.mean(aa_rast)), "lost_pixels": aa_lost,
               "fragments_per_frame": F_aa_mean, "fragments_found_with_skipping": float(np.mean(F_aa_proc)),
               "mask_evaluations": float(np.mean(aa_tests)), "triangles_skipped": float(np.mean(aa_skipped))},
        "roofline_aa": roofline_aa,
        "lenses": lens_stats,
        "wireframe": {"fps": 1e3 / (np.mean(w_map) + np.mean(w_bin) + np.mean(w_rast)),
                      "map_ms": float(np.mean(w_map)), "bin_ms": float(np.mean(w_bin)),
                      "raster_ms": float(np.mean(w_rast))},
        "roofline_wire": roofline_wire,
        "particles": {"fps": 1e3 / (np.mean(p_map) + np.mean(p_bin) + np.mean(p_rast)),
                      "setup_ms": float(np.mean(p_setup)), "map_ms": float(np.mean(p_map)),
                      "bin_ms": float(np.mean(p_bin)), "raster_ms": float(np.mean(p_rast)),
                      "fragments_found_with_skipping": part_found, "mask_evaluations": part_evals,
                      "lost_pixels": part_lost},
        "roofline_particles": roofline_particles,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
