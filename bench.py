#!/usr/bin/env python3
"""Frame-rate bench of the per-frame rendering path on one MI355X.

Workload (synthetic, seeded): 20M points from 4 simulated scans of a 40 x 30 x 6 m
multi-room scene (1 m grid cells), a 120-frame orbit camera path at 1920x1080
(90 degree horizontal fov), depth filter with 5 levels and filter_strength 0.5,
U-Net with widths 32/64/128/256 and He-initialised weights.

One step = one frame of the whole path: cull + splat + resolve (lnr_render),
depth filter (lnr_depth_filter) and U-Net (lnr_reconstruct), with the cloud
and weights already resident in HBM.  `value` is float32-U-Net frames/s; the
bfloat16 modes are reported beside it with their error against the float64
oracle on sampled windows.  Prints one JSON line on stdout.

    python bench.py [--gpus 1] [--steps 120] [--warmup 10]
"""

from __future__ import annotations

import argparse
import contextlib
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "frames/s and p50/p99 latency at 1080p/20M pts; BF16 vs FP32 U-Net at stated PSNR"
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0, "fp8": 5000.0}
TOL = {"fp32": 1e-4, "bf16": 2e-2, "bf16x3": 2e-2, "fp16": 2e-2, "fp8": 8e-2, "fp8x3": 8e-2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def conv_shapes(widths, H, W, cin0):
    """(name, H_l, W_l, c_out, c_in) of every 3x3 convolution, with the logical c_in."""
    L = len(widths)
    out = []
    for l in range(L):
        out.append((f"conv/enc{l}a", H >> l, W >> l, widths[l], 5 if l == 0 else widths[l - 1]))
        out.append((f"conv/enc{l}b", H >> l, W >> l, widths[l], widths[l]))
    for l in range(L - 2, -1, -1):
        out.append((f"conv/dec{l}a", H >> l, W >> l, widths[l], widths[l] + widths[l + 1]))
        out.append((f"conv/dec{l}b", H >> l, W >> l, widths[l], widths[l]))
    return out


RENDER_KERNELS = ("clear", "cull", "bin", "tilescan", "segsort", "tile", "tileres", "splat", "resolve")
FILTER_KERNELS = ("pyramid", "upsample")


def algorithmic_bytes(H, W, n_levels, n_proc, n_filled, n_removed):
    """Bytes the geometric stages must move (reads + writes) per frame: the
    projection reads 12 B per processed point (xyz) and writes 16 B per pixel
    (key, depth, rgba) plus a 4 B colour read per filled pixel; the pyramid
    reads 8 B per pixel (depth, rgba) and writes 4 B per pixel of every
    coarser level; the fused upsample reads 8 B per pixel and 4 B per pixel of
    every coarser level and writes 8 B per removed pixel.  Intermediate
    buffers an implementation adds (z-buffer clears, binned records) are not
    algorithmic."""
    P = H * W
    sizes = [(H, W)]
    for _ in range(n_levels):
        h, w = sizes[-1]
        sizes.append(((h + 1) // 2, (w + 1) // 2))
    px = [h * w for h, w in sizes]
    coarse = 4 * sum(px[1:])
    return {
        "render": 12 * n_proc + 16 * P + 4 * n_filled,
        "pyramid": 8 * P + coarse,
        "upsample": 8 * P + coarse + 8 * n_removed,
        "bin": 12 * n_proc,
    }


def host_info():
    info = {"host": platform.node(), "nproc": os.cpu_count()}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        info["rocm"] = open("/opt/rocm/.info/version").read().strip()
    except OSError:
        pass
    return info


_GEO = {}


def _geo_frame(i):
    """One frame's oracle projection + resolve + depth filter in a forked worker
    (one thread); the grid and cameras come from the parent through fork."""
    from oracle import depth_filter as F
    from oracle import render as R
    g, cams, n_levels, fs = _GEO["g"], _GEO["cams"], _GEO["n_levels"], _GEO["fs"]
    cam = cams[i % len(cams)]
    _, depth, rgba = R.render(g, cam)
    F.depth_filter(depth.reshape(cam.height, cam.width), rgba.reshape(cam.height, cam.width, 4), n_levels, fs)
    return i


def cpu_geometry_all_cores(scene, cams, n_levels, fs):
    """The oracle's projection + resolve + depth filter, one frame per host
    core at once (forked worker processes, numpy single-threaded, at most 15
    of them).  Called before the process touches the GPU, so the workers fork
    from a process without a device context.  Returns the oracle grid (reused
    by cpu_baseline) and the leg."""
    import multiprocessing as mp
    from oracle import grid as G
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    g = G.partition(scene.xyz, scene.rgb, 1.0)
    try:
        ncores = max(1, min(len(os.sched_getaffinity(0)), 15, len(cams)))
        _GEO.update(g=g, cams=cams, n_levels=n_levels, fs=fs)
        one_thread = threadpool_limits(limits=1) if threadpool_limits is not None else contextlib.nullcontext()
        with one_thread, mp.get_context("fork").Pool(ncores) as pool:
            t0 = time.perf_counter()
            pool.map(_geo_frame, range(ncores), chunksize=1)
            t = time.perf_counter() - t0
        leg = {"frames": ncores, "processes": ncores, "wall_s": round(t, 3), "frames_per_s": round(ncores / t, 3)}
    except Exception as e:  # pragma: no cover - a host without fork
        leg = {"error": str(e)}
    finally:
        _GEO.clear()
    return g, leg


def cpu_baseline(scene, cams, blob, n_levels, fs, widths, pre=None):
    """The CPU oracle as it stands, on a bounded sample of the workload: the
    projection + resolve + depth filter of frame 0 over all points (numpy, one
    thread), the same for one frame per core in forked single-threaded workers
    (the all-core rate of the geometric part, measured beforehand by
    cpu_geometry_all_cores: pre = its result), and the float64 U-Net on a
    centre crop, once with one BLAS thread and once with every core, scaled by
    pixel count to the full frame (a full 1080p frame takes several minutes in
    float64, so the U-Net leg is extrapolated and flagged as such)."""
    cam = cams[0]
    import numpy as np
    from oracle import depth_filter as F
    from oracle import grid as G
    from oracle import render as R
    from oracle import unet as U
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        all_threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        threadpool_limits, all_threads = None, 1
    g, geo_all = pre if pre is not None else (G.partition(scene.xyz, scene.rgb, 1.0), None)
    t0 = time.perf_counter()
    _, depth, rgba = R.render(g, cam)
    H, W = cam.height, cam.width
    fd, fr, _ = F.depth_filter(depth.reshape(H, W), rgba.reshape(H, W, 4), n_levels, fs)
    t_geo = time.perf_counter() - t0
    net = U.parse_blob(blob)

    def unet_crop(c):
        y0, x0 = H // 2 - c // 2, W // 2 - c // 2
        t = time.perf_counter()
        U.forward(net, fd[y0:y0 + c, x0:x0 + c], fr[y0:y0 + c, x0:x0 + c])
        return time.perf_counter() - t

    c_all, c_one = 256, 96
    t_all = unet_crop(c_all)
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t_one = unet_crop(c_one)
    else:  # pragma: no cover
        t_one = float("nan")
    s_all = t_all * (H * W) / (c_all * c_all)
    s_one = t_one * (H * W) / (c_one * c_one)
    return {
        "value": round(1.0 / (t_geo + s_all), 6), "unit": "frames/s", "cores": int(all_threads), "kind": "oracle",
        "extrapolated": True,
        "sample": (f"frame 0 of the path: oracle projection + resolve + depth filter over all {scene.n} points "
                   f"({t_geo:.2f} s measured, one thread), plus the float64 U-Net on a {c_all}x{c_all} centre crop "
                   f"({t_all:.2f} s with {all_threads} BLAS threads) scaled by pixel count to {W}x{H} "
                   f"({s_all:.1f} s extrapolated)"),
        "seconds_per_frame": round(t_geo + s_all, 3),
        "legs": {"geometry_s": round(t_geo, 3), "geometry_threads": 1, "geometry_all_cores": geo_all,
                 "unet_all_cores_s": round(s_all, 1), "unet_all_cores_threads": int(all_threads),
                 "unet_all_cores_crop": c_all,
                 "unet_one_thread_s": round(s_one, 1), "unet_one_thread_crop": c_one,
                 "frames_per_s_one_thread": round(1.0 / (t_geo + s_one), 6)},
    }


def parity_every_10th(L, ctx, cloud, net_fp32, cams, g, blob, H, W, n_levels, fs, progress=None):
    """Parity along the path, outside the timed region: every 10th frame's key,
    depth and rgba after the projection and the depth filter bit for bit
    against the oracle, and the fp32 U-Net on one seeded 64x64 window of each
    against the float64 oracle (computed on a crop grown by the receptive
    margin)."""
    import numpy as np
    import torch
    from oracle import depth_filter as F
    from oracle import render as R
    from oracle import unet as U
    net = U.parse_blob(blob)
    rng = np.random.default_rng(10)
    img = L.Image(H, W)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    frames, bad, max_abs = [], [], 0.0
    for i in range(0, len(cams), 10):
        cam = cams[i]
        L.lnr_render(ctx, cloud, cam, img)
        key = img.key.cpu().numpy().view(np.uint64).copy()
        L.lnr_depth_filter(ctx, img, n_levels, fs)
        L.lnr_reconstruct(ctx, net_fp32, img, out)
        torch.cuda.synchronize()
        d, r = img.depth.cpu().numpy(), img.rgba.cpu().numpy()
        k_ref, depth, rgba = R.render(g, cam)
        fd, fr, _ = F.depth_filter(depth.reshape(H, W), rgba.reshape(H, W, 4), n_levels, fs)
        if not (np.array_equal(key, k_ref.reshape(-1)) and np.array_equal(d.view(np.uint32), fd.view(np.uint32))
                and np.array_equal(r, fr)):
            bad.append(i)
        y0, x0 = int(rng.integers(0, H - 64)), int(rng.integers(0, W - 64))
        ref = U.forward_crop(net, fd, fr, y0, y0 + 64, x0, x0 + 64)
        e = float(np.abs(out[:, y0:y0 + 64, x0:x0 + 64].cpu().numpy().astype(np.float64) - ref).max())
        max_abs = max(max_abs, e)
        frames.append(i)
        if progress is not None:
            progress(f"parity frame {i}: projection and filter {'bit-exact' if i not in bad else 'DIFFER'}, "
                     f"fp32 U-Net window max-abs {e:.2e}")
    return {"frames": frames, "projection_and_filter_bit_exact": not bad, "frames_differing": bad,
            "unet_fp32_window_max_abs": max_abs, "unet_fp32_bound": TOL["fp32"],
            "unet_fp32_within_bound": max_abs <= TOL["fp32"]}


def sampled_error(fd, fr, blob, outs, H, W, progress=None, tol=None):
    """max-abs and PSNR of each precision's output against the float64 oracle on
    three 64x64 windows (centre, a corner, an edge), each computed on a crop
    grown by the receptive margin so the values equal the full-frame ones.
    `tol` maps a precision to its max-abs bound (default: TOL)."""
    import numpy as np
    from oracle import metrics as M
    from oracle import unet as U
    net = U.parse_blob(blob)
    wins = [(H // 2 - 32, H // 2 + 32, W // 2 - 32, W // 2 + 32), (0, 64, 0, 64), (H - 64, H, W // 3, W // 3 + 64)]
    refs = []
    for k, w in enumerate(wins):
        refs.append(U.forward_crop(net, fd, fr, *w))
        if progress is not None:
            progress(f"oracle window {k + 1}/{len(wins)} done")
    tol = TOL if tol is None else tol
    res = {}
    for name, y in outs.items():
        got = np.concatenate([y[:, a:b, c:d].reshape(3, -1) for (a, b, c, d) in wins], axis=1)
        ref = np.concatenate([r.reshape(3, -1) for r in refs], axis=1)
        res[name] = {"max_abs": M.max_abs(got, ref), "psnr_db": round(M.psnr(got, ref), 2),
                     "bound": tol[name], "within_bound": bool(M.max_abs(got, ref) <= tol[name])}
    return res


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_unet_fp32_multiroom_1080p.json")
TRAFFIC_SOURCES = [os.path.join(ROOT, "paper_2502_11618_amd", "csrc", f) for f in ("unet.hip", "api.cpp")]


def _sources_sha():
    import hashlib
    h = hashlib.sha256()
    for path in TRAFFIC_SOURCES:
        h.update(open(path, "rb").read())
    return h.hexdigest()


def summarize_counters(args):
    """Per-kernel HBM bytes from rocprofv3 --pmc csv files of a float32 frames
    run, each counter scaled by what it reads for a plain 1 GiB device copy.
    Convolutions are named by their place in the frame (a frame's first
    convolution is the one that stages the RGBDA image, or follows the input
    pack; the n-th after it is the n-th layer of conv_shapes), so the figures
    stay tied to layers whatever template a layer dispatches to.
    Writes every layer's figures next to the hash of the sources that decide
    them."""
    import collections
    import csv

    widths = (32, 64, 128, 256)
    layer_names = [n for (n, *_rest) in conv_shapes(widths, 1080, 1920, 8)]

    def rows(path):
        return sorted(csv.DictReader(open(path)), key=lambda r: int(r["Dispatch_Id"]))

    def mean(v):
        return sum(v) / len(v)

    def short(name):
        return name.replace("lnr::(anonymous namespace)::", "").replace("void ", "").split("(")[0]

    gib_kib = (1 << 30) / 1024.0
    f_fac = gib_kib / mean([float(r["Counter_Value"]) for r in rows(args.copy_fetch_csv)
                            if "copyBuffer" in r["Kernel_Name"]])
    w_fac = gib_kib / mean([float(r["Counter_Value"]) for r in rows(args.copy_write_csv)
                            if "copyBuffer" in r["Kernel_Name"]])
    per = collections.OrderedDict()
    kname = {}
    for path, key, fac in ((args.fetch_csv, "fetch", f_fac), (args.write_csv, "write", w_fac)):
        conv_i = None
        for r in rows(path):
            name = short(r["Kernel_Name"])
            if name.startswith("pack_kernel"):
                conv_i = 0
            if name.startswith("conv3x3") and name.endswith(", true>"):
                conv_i = 0  # the first convolution stages the RGBDA image itself
            if name.startswith(("conv3x3", "wino3x3")) and conv_i is not None and conv_i < len(layer_names):
                kname[layer_names[conv_i]] = name
                name = layer_names[conv_i]
                conv_i += 1
            per.setdefault(name, {"fetch": [], "write": []})[key].append(float(r["Counter_Value"]) * fac * 1024)
    print(f"counter scale factors from a 1 GiB copy: FETCH_SIZE x{f_fac:.4f}, WRITE_SIZE x{w_fac:.4f}")
    print(f"{'kernel':36s} {'template':34s} {'dispatches':>10s} {'fetch MB':>10s} {'write MB':>10s}")
    layers = {}
    for name, d in per.items():
        if not d["fetch"]:
            continue
        f, w = mean(d["fetch"]), (mean(d["write"]) if d["write"] else 0.0)
        print(f"{name:36s} {kname.get(name, ''):34s} {len(d['fetch']):10d} {f / 1e6:10.2f} {w / 1e6:10.2f}")
        if name.startswith("conv/"):
            layers[name] = {"template": kname[name], "fetch_bytes": f, "write_bytes": w}
    out = {"workload": "multiroom-20M-pts-1920x1080-orbit120, float32 U-Net 32/64/128/256", "layers": layers,
           "fetch_scale": f_fac, "write_scale": w_fac, "sources_sha256": _sources_sha()}
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"per-layer HBM bytes -> {TRAFFIC_JSON}")


def recorded_traffic(kernel):
    """HBM bytes per launch of the float32 layer `kernel` from the committed
    counter summary, or None when the sources that decide it changed since."""
    try:
        t = json.load(open(TRAFFIC_JSON))
    except (OSError, ValueError):
        return None
    if t.get("sources_sha256") != _sources_sha() or kernel not in t.get("layers", {}):
        return None
    lay = t["layers"][kernel]
    return lay["fetch_bytes"] + lay["write_bytes"]


def serve_bench(L, scene, cloud, blob, seconds, n_sessions=64, seed=0, budget=32 << 30, max_batch=8, lanes=2):
    """Serving: n_sessions viewers with seeded random-walk cameras at resolutions
    drawn from {640x480, 1280x720, 1920x1080}, Poisson arrivals at U(30, 90) Hz
    per session, fp16 U-Net (the 16-bit mode within the 2e-2 bound; plain bf16
    runs at the same speed but misses it), admitted under an HBM budget; continuous batching
    of same-resolution requests across sessions.  Latency = host time from
    submit to the poll that sees the frame finished; a request replaced by a
    newer camera of its session before it ran is superseded, and its wait
    (submit to the poll that reports it) is reported separately."""
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    sizes = [(640, 480), (1280, 720), (1920, 1080)]
    sctx = L.lnr_context_create(0, budget)
    net = L.lnr_unet_load(sctx, blob, L.LNR_FP16)
    srv = L.lnr_server_create(sctx, cloud, net, max_batch=max_batch, lanes=lanes, n_levels=5, filter_strength=0.5,
                              use_graphs=True, max_width=1920, max_height=1080)
    sess = []
    refused = 0
    for i in range(n_sessions):
        w, h = sizes[int(rng.integers(3))]
        rate = float(rng.uniform(30.0, 90.0))
        try:
            sid = L.lnr_server_open_session(srv, w, h)
        except L.LnrError as e:
            if e.status != L.LNR_E_BUDGET:
                raise
            refused += 1
            continue
        n_frames = int(rate * seconds * 1.5) + 8
        cams = [L.camera_struct(c) for c in synth.random_walk_path(scene, n_frames, seed=1000 + i, width=w, height=h)]
        sess.append({"sid": sid, "w": w, "h": h, "rate": rate, "cams": cams, "k": 0,
                     "next": float(rng.exponential(1.0 / rate))})
    submit_t = {}
    lat, sup_wait, batches, per_res = [], [], [], {}
    submitted = 0
    t0 = time.perf_counter()
    tag = 0

    def drain_results(now):
        for r in L.lnr_server_poll(srv):
            t_sub, res = submit_t.pop(r["tag"])
            if r["superseded"]:
                sup_wait.append(now - t_sub)
                continue
            lat.append(now - t_sub)
            batches.append(r["batch"])
            per_res[res] = per_res.get(res, 0) + 1

    while True:
        now = time.perf_counter() - t0
        if now >= seconds:
            break
        for ss in sess:
            while ss["next"] <= now and ss["k"] < len(ss["cams"]):
                L.lnr_server_submit(srv, ss["sid"], ss["cams"][ss["k"]], tag)
                submit_t[tag] = (time.perf_counter() - t0, f"{ss['w']}x{ss['h']}")
                tag += 1
                submitted += 1
                ss["k"] += 1
                ss["next"] += float(rng.exponential(1.0 / ss["rate"]))
        while L.lnr_server_step(srv) > 0:
            pass
        drain_results(time.perf_counter() - t0)
    t_end = time.perf_counter() - t0
    for _ in range(1000000):
        L.lnr_server_step(srv)
        drain_results(time.perf_counter() - t0)
        pend, infl = L.lnr_server_pending(srv)
        if pend == 0 and infl == 0 and not submit_t:
            break
    elapsed = time.perf_counter() - t0
    lat_ms = np.array(lat) * 1000.0
    sup_ms = np.array(sup_wait) * 1000.0
    done = len(lat)
    px = sum(int(k.split("x")[0]) * int(k.split("x")[1]) * v for k, v in per_res.items())

    def pct(v, q):
        return round(float(np.percentile(v, q)), 3) if len(v) else None

    L.lnr_server_destroy(srv)
    return {
        "sessions": n_sessions, "sessions_admitted": len(sess), "sessions_refused": refused,
        "seconds_of_arrivals": round(t_end, 2), "offered_requests_per_s": round(submitted / t_end, 1),
        "requests": submitted, "completed": done, "superseded": len(sup_wait),
        "superseded_fraction": round(len(sup_wait) / max(1, submitted), 4),
        "frames_per_s": round(done / elapsed, 1), "megapixels_per_s": round(px / elapsed / 1e6, 1),
        "latency_ms": {"p50": pct(lat_ms, 50), "p99": pct(lat_ms, 99)},
        "superseded_wait_ms": {"p50": pct(sup_ms, 50), "p99": pct(sup_ms, 99)},
        "mean_batch": round(float(np.mean(batches)), 2) if batches else None,
        "frames_by_resolution": per_res, "budget_bytes": budget, "max_batch": max_batch, "lanes": lanes,
        "precision": "fp16",
    }


def serve_sweep(L, scene, cloud, blob, seconds, counts=(8, 16, 32, 64)):
    """The serving workload at several session counts (the same seeded
    sessions, the first n of them): throughput, latency and superseded
    fraction against offered load."""
    out = []
    for n in counts:
        r = serve_bench(L, scene, cloud, blob, seconds, n_sessions=n)
        log(f"serving {n} sessions: {r['frames_per_s']} frames/s of {r['offered_requests_per_s']} requests/s offered, "
            f"superseded {100 * r['superseded_fraction']:.1f}%, p50 {r['latency_ms']['p50']} ms, "
            f"p99 {r['latency_ms']['p99']} ms")
        out.append(r)
    return out


def multiview_render(L, ctx, cloud, cams, W, H, batch, nbatch):
    """Projection of one batch of views, view by view (the default tiled splat,
    each view reading its visible cells' points) against lnr_render_views (one
    pass per 8 views, each point of a cell visible in any of them read once):
    time per batch by HIP events on the stream both run on, points read, and
    whether every image is the same bit for bit."""
    import numpy as np
    import torch

    imgs = [L.Image(H, W) for _ in range(batch)]
    ref = [L.Image(H, W) for _ in range(batch)]
    single_ms, multi_ms, read_single, read_multi, same = [], [], [], [], True
    for b in range(1 + nbatch):  # batch 0 warms up
        bc = [cams[(b * batch + v) % len(cams)] for v in range(batch)]
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for v in range(batch):
            L.lnr_render(ctx, cloud, bc[v], ref[v])
        e[1].record()
        L.lnr_render_views(ctx, cloud, bc, imgs)
        e[2].record()
        torch.cuda.synchronize()
        if b == 0:
            continue
        single_ms.append(e[0].elapsed_time(e[1]))
        multi_ms.append(e[1].elapsed_time(e[2]))
        read_multi.append(L.lnr_render_stats(ctx)[1])
        n = 0
        for v in range(batch):
            L.lnr_render(ctx, cloud, bc[v], ref[v])
            torch.cuda.synchronize()
            n += L.lnr_render_stats(ctx)[1]
        read_single.append(n)
        same = same and all(torch.equal(imgs[v].key, ref[v].key) and torch.equal(imgs[v].depth, ref[v].depth)
                            and torch.equal(imgs[v].rgba, ref[v].rgba) for v in range(batch))
    return {"views_per_batch": batch, "batches": nbatch,
            "view_by_view_ms_per_batch": round(float(np.mean(single_ms)), 3),
            "multi_view_ms_per_batch": round(float(np.mean(multi_ms)), 3),
            "points_read_view_by_view": int(np.mean(read_single)),
            "points_read_multi_view": int(np.mean(read_multi)),
            "images_identical": bool(same)}


def largest_scene(args):
    """The largest configuration: 300M points from 16 scans of an 80 x 60 x 10 m
    scene of 32 rooms (2 m cells); batches of 8 consecutive orbit-path views at
    3840x2160; depth filter n = 6, fs = 0.5; U-Net widths 32/64/128/256/512 in
    fp32, fp16, split bf16, bf16, split e4m3 and e4m3, each held to its own
    bound (e4m3: 8e-2).  A batch renders, filters and reconstructs its
    8 views one after the other into 8 output images (a 4K view fills the GPU
    on its own).  Reports views/s, batch time, per-view latency, the U-Net's
    share against the matrix peak and the sampled error of view 0 against the
    float64 oracle.  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2502_11618_amd as L
    import synth

    W, H, FOV, NL, FS, CELL, BATCH, NBATCH = 3840, 2160, 90.0, 6, 0.5, 2.0, 8, 3
    widths = (32, 64, 128, 256, 512)
    t0 = time.perf_counter()
    scene = synth.scene_for_config("huge", seed=0, cache=False, progress=log)
    log(f"scene {scene.name}: {scene.n} points ({time.perf_counter() - t0:.1f} s)")
    blob = synth.make_unet_blob(widths, seed=0)
    ctx = L.lnr_context_create(0)
    t0 = time.perf_counter()
    cloud = L.lnr_cloud_load(ctx, scene.xyz, scene.rgb, CELL)
    load_s = time.perf_counter() - t0
    info = L.lnr_cloud_info(cloud)
    log(f"cloud loaded and partitioned in {load_s:.2f} s, grid {info['dims']}")
    cams = synth.orbit_path(scene, 120, W, H, FOV)
    prec_ids = {"fp32": L.LNR_FP32, "fp16": L.LNR_FP16, "bf16x3": L.LNR_BF16X3, "bf16": L.LNR_BF16,
                "fp8x3": L.LNR_FP8_E4M3X3, "fp8": L.LNR_FP8_E4M3}
    mv = multiview_render(L, ctx, cloud, cams, W, H, BATCH, NBATCH)
    log(f"projection of a batch of {BATCH}: view by view {mv['view_by_view_ms_per_batch']} ms "
        f"({mv['points_read_view_by_view']} points read), multi-view {mv['multi_view_ms_per_batch']} ms "
        f"({mv['points_read_multi_view']} points read), identical: {mv['images_identical']}")
    if args.projection_only:
        print(json.dumps({"mode": "largest", "workload": "huge-300M-pts-16-scans-8x4K-batches", "points": scene.n,
                          "multi_view_render": mv, "env": host_info()}), flush=True)
        return
    nets = {p: L.lnr_unet_load(ctx, blob, i) for p, i in prec_ids.items()}
    img = L.Image(H, W)
    outs = [torch.empty((3, H, W), dtype=torch.float32, device="cuda") for _ in range(BATCH)]

    def run_batch(b, net, ev=None):
        for v in range(BATCH):
            if ev is not None:
                ev[v][0].record()
            L.lnr_render(ctx, cloud, cams[(b * BATCH + v) % len(cams)], img)
            L.lnr_depth_filter(ctx, img, NL, FS)
            L.lnr_reconstruct(ctx, net, img, outs[v])
            if ev is not None:
                ev[v][1].record()

    shapes = conv_shapes(widths, H, W, 8)
    unet_flops = sum(2.0 * h * w * co * 9 * ci for (_, h, w, co, ci) in shapes) + 2.0 * H * W * 3 * widths[0]
    # flops the matrix cores execute: fp32 layers past the first by Winograd
    # F(2x2, 3x3) (16 multiplies per 2x2 block and channel pair; the first
    # layer multiplies 6 of its 8 staged channels), three passes per product
    # in the split modes
    fp32_exec = sum((2.0 * ((h + 1) // 2) * ((w + 1) // 2) * 16 * co * ci if i > 0 else 2.0 * h * w * co * 9 * 6)
                    for i, (_, h, w, co, ci) in enumerate(shapes)) + 2.0 * H * W * 3 * widths[0]
    executed = {"fp32": fp32_exec, "bf16x3": 3.0 * unet_flops, "fp8x3": 3.0 * unet_flops}
    res = {}
    for p, net in nets.items():
        run_batch(0, net)
        torch.cuda.synchronize()
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(BATCH)]
              for _ in range(NBATCH)]
        t0 = time.perf_counter()
        for b in range(NBATCH):
            run_batch(1 + b, net, ev[b])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(e) for evb in ev for a, e in evb])
        # the U-Net alone, on the last view's image, for its share of the matrix peak
        ue = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for a, e in ue:
            a.record()
            L.lnr_reconstruct(ctx, net, img, outs[0])
            e.record()
        torch.cuda.synchronize()
        unet_ms = float(np.mean([a.elapsed_time(e) for a, e in ue]))
        peak = PEAK_TFLOPS["fp32" if p == "fp32" else ("fp8" if p.startswith("fp8") else "bf16")]
        res[p] = {"views_per_s": round(NBATCH * BATCH / wall, 2), "ms_per_batch": round(1000 * wall / NBATCH, 3),
                  "view_latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                                      "p99": round(float(np.percentile(lat, 99)), 3)},
                  "unet_ms": round(unet_ms, 3),
                  "unet_roofline": {"bound": "mfma", "achieved": round(executed.get(p, unet_flops) / (unet_ms * 1e-3) / 1e12, 2),
                                    "peak": peak, "unit": "TFLOP/s",
                                    "frac": round(executed.get(p, unet_flops) / (unet_ms * 1e-3) / 1e12 / peak, 4),
                                    "effective_tflops": round(unet_flops / (unet_ms * 1e-3) / 1e12, 2)}}
        log(f"{p}: {res[p]['views_per_s']} views/s, {res[p]['ms_per_batch']} ms per batch of {BATCH}, "
            f"U-Net {unet_ms:.2f} ms")
    proc = []
    for b in range(NBATCH):
        for v in range(BATCH):
            L.lnr_render(ctx, cloud, cams[((1 + b) * BATCH + v) % len(cams)], img)
            torch.cuda.synchronize()
            proc.append(L.lnr_render_stats(ctx)[1])
    L.lnr_render(ctx, cloud, cams[0], img)
    L.lnr_depth_filter(ctx, img, NL, FS)
    torch.cuda.synchronize()
    fd, fr = img.depth.cpu().numpy(), img.rgba.cpu().numpy()
    host = {}
    for p, net in nets.items():
        L.lnr_reconstruct(ctx, net, img, outs[0])
        torch.cuda.synchronize()
        host[p] = outs[0].cpu().numpy().astype(np.float64)
    err = sampled_error(fd, fr, blob, host, H, W, progress=log)
    for p in res:
        res[p]["error_vs_fp64_sampled"] = err[p]
    print(json.dumps({"mode": "largest", "workload": "huge-300M-pts-16-scans-8x4K-batches",
                      "points": scene.n, "cell_m": CELL, "grid_dims": list(info["dims"]),
                      "load_partition_s": round(load_s, 3), "width": W, "height": H, "batch_views": BATCH,
                      "timed_batches": NBATCH, "n_levels": NL, "filter_strength": FS, "unet_widths": list(widths),
                      "unet_flops_per_view": unet_flops,
                      "processed_points_per_view": {"mean": float(np.mean(proc)), "min": int(min(proc)),
                                                    "max": int(max(proc))},
                      "multi_view_render": mv, "results": res, "env": host_info()}), flush=True)


def precision_tier(args, scene_name="large", n_points=None, sizes=((1920, 1080), (2560, 1440)),
                   workload="large-100M-pts-8-scans-orbit", mode="precision-tier"):
    """The precision tier on the larger scene: 100M points from 8 scans (1 m
    cells), 60 frames of the orbit path at 1920x1080 and at 2560x1440, depth
    filter n = 5, fs = 0.5, U-Net 32/64/128/256 in fp32, fp16, split bf16,
    bf16, split e4m3 and e4m3:
    frames/s, per-frame latency and the sampled error against the float64
    oracle of each precision.  With other arguments, the same run on another
    scene and other image sizes (the paper's Table 1 shapes: the multi-room
    generator at 23M points, 1920x1440 and 960x720).  Prints one JSON line."""
    import numpy as np
    import torch
    import paper_2502_11618_amd as L
    import synth

    FOV, NL, FS, STEPS = 90.0, 5, 0.5, 60
    widths = (32, 64, 128, 256)
    t0 = time.perf_counter()
    scene = synth.scene_for_config(scene_name, seed=0, n_points=n_points)
    log(f"scene {scene.name}: {scene.n} points ({time.perf_counter() - t0:.1f} s)")
    blob = synth.make_unet_blob(widths, seed=0)
    ctx = L.lnr_context_create(0)
    t0 = time.perf_counter()
    cloud = L.lnr_cloud_load(ctx, scene.xyz, scene.rgb, 1.0)
    load_s = time.perf_counter() - t0
    prec_ids = {"fp32": L.LNR_FP32, "fp16": L.LNR_FP16, "bf16x3": L.LNR_BF16X3, "bf16": L.LNR_BF16,
                "fp8x3": L.LNR_FP8_E4M3X3, "fp8": L.LNR_FP8_E4M3}
    nets = {p: L.lnr_unet_load(ctx, blob, i) for p, i in prec_ids.items()}
    out_all = {}
    for W, H in sizes:
        cams = synth.orbit_path(scene, 120, W, H, FOV)
        img = L.Image(H, W)
        out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
        res = {}
        for p, net in nets.items():
            for i in range(5):
                L.lnr_render(ctx, cloud, cams[i], img)
                L.lnr_depth_filter(ctx, img, NL, FS)
                L.lnr_reconstruct(ctx, net, img, out)
            torch.cuda.synchronize()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(STEPS)]
            t0 = time.perf_counter()
            for i in range(STEPS):
                ev[i][0].record()
                L.lnr_render(ctx, cloud, cams[2 * i], img)
                L.lnr_depth_filter(ctx, img, NL, FS)
                L.lnr_reconstruct(ctx, net, img, out)
                ev[i][1].record()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            lat = np.array([a.elapsed_time(b) for a, b in ev])
            res[p] = {"frames_per_s": round(STEPS / wall, 2), "ms_per_frame": round(1000 * wall / STEPS, 4),
                      "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                                     "p99": round(float(np.percentile(lat, 99)), 4)}}
        L.lnr_render(ctx, cloud, cams[0], img)
        L.lnr_depth_filter(ctx, img, NL, FS)
        torch.cuda.synchronize()
        _, proc, _ = L.lnr_render_stats(ctx)
        fd, fr = img.depth.cpu().numpy(), img.rgba.cpu().numpy()
        outs = {}
        for p, net in nets.items():
            L.lnr_reconstruct(ctx, net, img, out)
            torch.cuda.synchronize()
            outs[p] = out.cpu().numpy().astype(np.float64)
        err = sampled_error(fd, fr, blob, outs, H, W)
        for p in res:
            res[p]["error_vs_fp64_sampled"] = err[p]
        out_all[f"{W}x{H}"] = {"processed_points_frame0": proc, "precisions": res}
        log(f"{W}x{H}: " + ", ".join(f"{p} {r['frames_per_s']} f/s" for p, r in res.items()))
    print(json.dumps({"mode": mode, "workload": workload,
                      "points": scene.n, "cell_m": 1.0, "load_partition_s": round(load_s, 3), "n_levels": NL,
                      "filter_strength": FS, "unet_widths": list(widths), "steps": STEPS, "results": out_all,
                      "env": host_info()}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=120)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--points", type=int, default=20_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precisions", default="fp32,fp16,bf16x3,bf16,fp8x3,fp8")
    ap.add_argument("--no-error-check", action="store_true", help="skip the float64 error windows")
    ap.add_argument("--pipelined", action="store_true",
                    help="overlap the next frame's projection and filter (second stream and context) with the "
                         "current frame's U-Net (default: frames one after the other on one stream)")
    ap.add_argument("--serve-seconds", type=float, default=3.0,
                    help="serving run length per session count of the sweep (0 = skip)")
    ap.add_argument("--mode", default="frames",
                    choices=["frames", "copy", "counters", "precision-tier", "paper-shapes", "largest"],
                    help="copy: only a plain 1 GiB device copy (calibrates HBM byte counters); "
                         "counters: summarise rocprofv3 FETCH_SIZE/WRITE_SIZE csv files (no GPU); "
                         "precision-tier: the 100M-point scene at 1080p and 1440p in every precision; "
                         "paper-shapes: the multi-room scene at 23M points, 1920x1440 and 960x720, every precision; "
                         "largest: the 300M-point scene, batches of 8 views at 3840x2160, 5-level U-Net")
    ap.add_argument("--projection-only", action="store_true",
                    help="largest mode: stop after comparing view-by-view and multi-view projection")
    ap.add_argument("--fetch-csv", help="counters mode: FETCH_SIZE counter_collection.csv of a frames run")
    ap.add_argument("--write-csv", help="counters mode: WRITE_SIZE counter_collection.csv of a frames run")
    ap.add_argument("--copy-fetch-csv", help="counters mode: FETCH_SIZE csv of a copy run")
    ap.add_argument("--copy-write-csv", help="counters mode: WRITE_SIZE csv of a copy run")
    args = ap.parse_args()
    if args.mode == "counters":
        summarize_counters(args)
        return
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU (asked for {args.gpus}); this build measures the one-GPU "
              "path only (frames, views and sessions shard across GPUs without exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.mode == "precision-tier":
        precision_tier(args)
        return
    if args.mode == "paper-shapes":
        precision_tier(args, "multiroom", 23_000_000, ((1920, 1440), (960, 720)),
                       "multiroom-23M-pts-1920x1440-and-960x720-orbit", "paper-shapes")
        return
    if args.mode == "largest":
        largest_scene(args)
        return
    if args.mode == "copy":
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copy", "bytes_read_per_copy": x.numel() * 4, "bytes_written_per_copy": y.numel() * 4,
                          "copies": 5}), flush=True)
        return

    import paper_2502_11618_amd as L
    import synth

    W, H, FOV, NL, FS = 1920, 1080, 90.0, 5, 0.5
    widths = (32, 64, 128, 256)
    t0 = time.perf_counter()
    scene = synth.scene_for_config("multiroom", seed=0, n_points=args.points)
    log(f"scene {scene.name}: {scene.n} points ({time.perf_counter() - t0:.1f} s)")
    cams = synth.orbit_path(scene, 120, W, H, FOV)
    blob = synth.make_unet_blob(widths, seed=0)
    geo_pre = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle's projection and filter on every core ...")
        geo_pre = cpu_geometry_all_cores(scene, cams, NL, FS)

    torch.cuda.set_device(0)
    ctx = L.lnr_context_create(0)
    t0 = time.perf_counter()
    cloud = L.lnr_cloud_load(ctx, scene.xyz, scene.rgb, 1.0)
    load_s = time.perf_counter() - t0
    info = L.lnr_cloud_info(cloud)
    log(f"cloud loaded and partitioned in {load_s:.2f} s, grid {info['dims']}")
    prec_ids = {"fp32": L.LNR_FP32, "bf16": L.LNR_BF16, "bf16x3": L.LNR_BF16X3, "fp16": L.LNR_FP16,
                "fp8": L.LNR_FP8_E4M3, "fp8x3": L.LNR_FP8_E4M3X3}
    precs = [p for p in args.precisions.split(",") if p]
    nets = {p: L.lnr_unet_load(ctx, blob, prec_ids[p]) for p in precs}
    img = L.Image(H, W)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")

    def frame(i, net):
        L.lnr_render(ctx, cloud, cams[i % len(cams)], img)
        L.lnr_depth_filter(ctx, img, NL, FS)
        L.lnr_reconstruct(ctx, net, img, out)

    # Pipelined frames: frame i's projection and filter run on their own
    # stream (and context: a context's calls must not overlap on two streams)
    # while frame i - 1's U-Net runs on the U-Net stream; two RGBDA images
    # alternate, an image being re-rendered only after the U-Net that read it.
    if args.pipelined:
        ctx_geo = L.lnr_context_create(0)
        s_geo, s_net = torch.cuda.Stream(), torch.cuda.current_stream()
        imgs = [L.Image(H, W), L.Image(H, W)]
        ready = [torch.cuda.Event(), torch.cuda.Event()]
        done = [torch.cuda.Event(), torch.cuda.Event()]
        for e in done:
            e.record(s_net)

    def frame_pipelined(i, net, ev=None):
        g = i & 1
        s_geo.wait_event(done[g])
        if ev is not None:
            ev[0].record(s_geo)
        L.lnr_render(ctx_geo, cloud, cams[i % len(cams)], imgs[g], stream=s_geo)
        L.lnr_depth_filter(ctx_geo, imgs[g], NL, FS, stream=s_geo)
        ready[g].record(s_geo)
        s_net.wait_event(ready[g])
        L.lnr_reconstruct(ctx, net, imgs[g], out, stream=s_net)
        done[g].record(s_net)
        if ev is not None:
            ev[1].record(s_net)

    run_frame = frame_pipelined if args.pipelined else frame

    results = {}
    kernel_stats = {}
    for p in precs:
        net = nets[p]
        for i in range(args.warmup):
            run_frame(i, net)
            if args.pipelined:
                frame(i, net)  # the per-kernel pass below runs sequential frames
        torch.cuda.synchronize()
        # pass 1: frame rate and per-frame latency (one event pair per frame,
        # from the start of its projection to the end of its U-Net)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            if args.pipelined:
                frame_pipelined(i, net, ev[i])
            else:
                ev[i][0].record()
                frame(i, net)
                ev[i][1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([a.elapsed_time(b) for a, b in ev])
        # pass 2: the same frames with every kernel bracketed by events on its stream
        L.lnr_profile_enable(ctx, True)
        L.lnr_profile_read(ctx)
        n_proc_total = 0
        per_kernel = {}
        for i in range(args.steps):
            frame(i, net)
            if p == precs[0]:
                torch.cuda.synchronize()
                vis, proc, _ = L.lnr_render_stats(ctx)
                n_proc_total += proc
            for name, ms in L.lnr_profile_read(ctx):
                per_kernel.setdefault(name, []).append(ms)
        L.lnr_profile_enable(ctx, False)
        torch.cuda.synchronize()
        results[p] = {
            "frames_per_s": args.steps / wall,
            "ms_per_frame": 1000.0 * wall / args.steps,
            "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                           "max": float(lat.max())},
        }
        kernel_stats[p] = {k: (float(np.mean(v)), len(v)) for k, v in per_kernel.items()}
        if p == precs[0]:
            results[p]["processed_points_per_frame"] = n_proc_total / args.steps
        log(f"{p}: {results[p]['frames_per_s']:.1f} frames/s, p50 {results[p]['latency_ms']['p50']:.2f} ms, "
            f"p99 {results[p]['latency_ms']['p99']:.2f} ms")

    # per-frame statistics of the timed frames (an untimed pass): processed
    # points, filled pixels after projection and pixels kept by the filter
    per_frame = {"processed_points": [], "filled_pixels": [], "kept_pixels": []}
    for i in range(args.steps):
        L.lnr_render(ctx, cloud, cams[i % len(cams)], img)
        torch.cuda.synchronize()
        per_frame["processed_points"].append(int(L.lnr_render_stats(ctx)[1]))
        per_frame["filled_pixels"].append(int((img.rgba[..., 3] != 0).sum().item()))
        L.lnr_depth_filter(ctx, img, NL, FS)
        per_frame["kept_pixels"].append(int((img.rgba[..., 3] != 0).sum().item()))
    # frame 0 again, for the error windows and the byte counts
    L.lnr_render(ctx, cloud, cams[0], img)
    torch.cuda.synchronize()
    _, proc0, _ = L.lnr_render_stats(ctx)
    filled0 = int((img.rgba[..., 3] != 0).sum().item())
    L.lnr_depth_filter(ctx, img, NL, FS)
    torch.cuda.synchronize()
    kept0 = int((img.rgba[..., 3] != 0).sum().item())
    fd, fr = img.depth.cpu().numpy(), img.rgba.cpu().numpy()
    outs = {}
    for p in precs:
        L.lnr_reconstruct(ctx, nets[p], img, out)
        torch.cuda.synchronize()
        outs[p] = out.cpu().numpy().astype(np.float64)
    errors = {p: None for p in precs} if args.no_error_check else sampled_error(fd, fr, blob, outs, H, W)

    # z-buffer atomics: the timed frames again, projection only, counting the
    # atomics each splat issues; and the device's 64-bit atomicMin rate on a
    # buffer of the image's size (pseudo-random words, then contended words)
    n_atomics = []
    for i in range(args.steps):
        L.lnr_render(ctx, cloud, cams[i % len(cams)], img, L.LNR_RENDER_COUNT_ATOMICS)
        n_atomics.append(L.lnr_render_atomic_count(ctx))
    # the same frames projected with the atomic splat (for comparison), per kernel
    L.lnr_profile_enable(ctx, True)
    L.lnr_profile_read(ctx)
    per_kernel = {}
    for i in range(args.steps):
        L.lnr_render(ctx, cloud, cams[i % len(cams)], img, L.LNR_RENDER_ATOMIC_SPLAT)
        for name, ms in L.lnr_profile_read(ctx):
            per_kernel.setdefault(name, []).append(ms)
    L.lnr_profile_enable(ctx, False)
    atomic_ks = {k: (float(np.mean(v)), len(v)) for k, v in per_kernel.items()}
    atomic_rate, atomic_ops = L.lnr_measure_atomic_min(ctx, H * W, 0, 1 << 26)
    atomic_rate_contended, _ = L.lnr_measure_atomic_min(ctx, H * W, 1, 1 << 26)

    # rooflines.  The float32 layers past the first run as Winograd F(2x2, 3x3):
    # the matrix cores execute 16 multiplies per 2x2 output block and channel
    # pair instead of the direct convolution's 36, and the first layer
    # multiplies 6 of its 8 staged channels (3 k-pairs) per tap.  `frac` is the
    # executed flops' share of the matrix peak (how busy the matrix cores
    # are); `effective_tflops` is the direct convolution's algorithmic flops
    # per second, which a Winograd kernel can push past the peak.
    p0 = precs[0]
    ks = kernel_stats[p0]
    cin0 = 8
    shapes = conv_shapes(widths, H, W, cin0)
    flops = {name: 2.0 * h * w * co * 9 * ci for (name, h, w, co, ci) in shapes}
    mfma_flops = {name: (2.0 * ((h + 1) // 2) * ((w + 1) // 2) * 16 * co * ci if i > 0 else 2.0 * h * w * co * 9 * 6)
                  for i, (name, h, w, co, ci) in enumerate(shapes)}
    # the 16-bit modes run both first-level convolutions as one kernel (conv/enc0)
    flops["conv/enc0"] = flops["conv/enc0a"] + flops["conv/enc0b"]
    mfma_flops["conv/enc0"] = mfma_flops["conv/enc0a"] + mfma_flops["conv/enc0b"]
    head_flops = 2.0 * H * W * 3 * widths[0]

    def conv_roofline(kstats, prec, executed):
        conv_ms = {k: v[0] for k, v in kstats.items() if k.startswith("conv/")}
        dom = max(conv_ms, key=conv_ms.get)
        peak = PEAK_TFLOPS[prec]
        ex = executed[dom] / (conv_ms[dom] * 1e-3) / 1e12
        eff = flops[dom] / (conv_ms[dom] * 1e-3) / 1e12
        return dom, {"kernel": dom, "bound": "mfma", "achieved": round(ex, 2), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(ex / peak, 4), "flops_per_launch": executed[dom],
                     "avg_launch_ms": round(conv_ms[dom], 4),
                     "algorithm": "winograd F(2x2,3x3)" if executed[dom] != flops[dom] else "direct",
                     "algorithmic_flops_per_launch": flops[dom], "effective_tflops": round(eff, 2)}

    exec_fp32 = mfma_flops if p0 == "fp32" else flops
    dom, roofline = conv_roofline(ks, p0, exec_fp32)
    traffic = recorded_traffic(dom) if p0 == "fp32" else None
    roofline["traffic"] = None if traffic is None else round(traffic)
    unet_flops = sum(v for k, v in flops.items() if k != "conv/enc0") + head_flops
    n_proc = results[p0].get("processed_points_per_frame", proc0)
    gbytes = algorithmic_bytes(H, W, NL, n_proc, filled0, filled0 - kept0)

    def geo_roofline(kstats, names, nbytes):
        ms = sum(kstats[k][0] for k in names if k in kstats)
        gbs = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_frame": nbytes, "ms_per_frame": round(ms, 4),
                "kernels": [k for k in names if k in kstats]}

    rf_bytes = gbytes["render"] + gbytes["pyramid"] + gbytes["upsample"]
    rooflines = {
        "render_and_filter": geo_roofline(ks, RENDER_KERNELS + FILTER_KERNELS, rf_bytes),
        "render": geo_roofline(ks, RENDER_KERNELS, gbytes["render"]),
        "filter": geo_roofline(ks, FILTER_KERNELS, gbytes["pyramid"] + gbytes["upsample"]),
        "render_atomic_splat": geo_roofline(atomic_ks, RENDER_KERNELS, gbytes["render"]),
    }
    for k in ("bin", "pyramid", "upsample"):
        if k in ks:
            gbs = gbytes[k] / (ks[k][0] * 1e-3) / 1e9
            rooflines[k] = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                            "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_launch": gbytes[k],
                            "avg_launch_ms": round(ks[k][0], 4)}
    if "splat" in atomic_ks and n_atomics:
        rate = float(np.mean(n_atomics)) / (atomic_ks["splat"][0] * 1e-3)
        rooflines["splat_atomics"] = {
            "bound": "atomic", "achieved": round(rate, 1), "peak": round(atomic_rate, 1), "unit": "atomics/s",
            "frac": round(rate / atomic_rate, 4), "atomics_per_frame": round(float(np.mean(n_atomics)), 1),
            "peak_kind": f"measured: {atomic_ops} 64-bit atomicMin on pseudo-random words of a {W}x{H} buffer",
            "contended_peak": round(atomic_rate_contended, 1)}
    def peak_kind(p):  # the matrix peak of the operand type
        return "fp32" if p == "fp32" else ("fp8" if p.startswith("fp8") else "bf16")

    for p in precs:
        kp = kernel_stats[p]
        ms = sum(v[0] for k, v in kp.items() if k.startswith("conv/") or k in ("pack", "head"))
        peak = PEAK_TFLOPS[peak_kind(p)]
        if p == "fp32":
            ex = sum(v for k, v in mfma_flops.items() if k != "conv/enc0") + head_flops
        elif p in ("bf16x3", "fp8x3"):
            ex = 3.0 * unet_flops  # three passes per product
        else:
            ex = unet_flops
        rooflines[f"unet_{p}_all_convs"] = {
            "bound": "mfma", "achieved": round(ex / (ms * 1e-3) / 1e12, 2), "peak": peak, "unit": "TFLOP/s",
            "frac": round(ex / (ms * 1e-3) / 1e12 / peak, 4), "executed_flops_per_frame": ex,
            "effective_tflops": round(unet_flops / (ms * 1e-3) / 1e12, 2), "ms_per_frame": round(ms, 4)}
        if p != p0:
            rooflines[f"dominant_{p}_kernel"] = conv_roofline(kp, peak_kind(p),
                                                              {k: (3.0 * v if p in ("bf16x3", "fp8x3") else v)
                                                               for k, v in flops.items()})[1]

    fps = results[p0]["frames_per_s"]
    line = {
        "metric": METRIC,
        "value": round(fps, 3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(results[p0]["ms_per_frame"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "multiroom-20M-pts-1920x1080-orbit120", "points": scene.n, "scans": 4,
                   "cell_m": 1.0, "width": W, "height": H, "fov_deg": FOV, "n_levels": NL, "filter_strength": FS,
                   "unet_widths": list(widths), "path_frames": len(cams), "timed_frames": args.steps,
                   "grid_dims": list(info["dims"]), "pipelined": bool(args.pipelined)},
        "latency_ms": {k: round(v, 4) for k, v in results[p0]["latency_ms"].items()},
        "points_per_s": round(n_proc * fps, 1),
        "points_per_s_projection": round(n_proc / (sum(ks[k][0] for k in RENDER_KERNELS if k in ks) * 1e-3), 1),
        "processed_points_per_frame": round(n_proc, 1),
        "precisions": {p: {"frames_per_s": round(r["frames_per_s"], 3), "ms_per_frame": round(r["ms_per_frame"], 4),
                           "latency_ms": {k: round(v, 4) for k, v in r["latency_ms"].items()},
                           "error_vs_fp64_sampled": errors[p]} for p, r in results.items()},
        "half_precision_within_bound": {
            p: {"frames_per_s": round(results[p]["frames_per_s"], 3), "max_abs": errors[p]["max_abs"],
                "bound": errors[p]["bound"]}
            for p in precs if p != "fp32" and errors.get(p) and errors[p]["within_bound"]},
        "stage_ms": {p: {k: round(v[0], 4) for k, v in sorted(kernel_stats[p].items())} for p in precs},
        "roofline": roofline,
        "rooflines": rooflines,
        "load_partition_s": round(load_s, 3),
        "frame0": {"processed_points": proc0, "filled_pixels": filled0, "kept_after_filter": kept0},
        "per_frame": per_frame,
        "env": host_info(),
    }
    if not args.no_error_check and "fp32" in nets:
        log("parity of every 10th frame of the path against the oracle ...")
        g_or = geo_pre[0] if geo_pre is not None else None
        if g_or is None:
            from oracle import grid as G
            g_or = G.partition(scene.xyz, scene.rgb, 1.0)
        line["parity_every_10th_frame"] = parity_every_10th(L, ctx, cloud, nets["fp32"], cams, g_or, blob, H, W,
                                                            NL, FS, progress=log)
    try:
        line["env"]["gpu"] = torch.cuda.get_device_name(0)
        line["env"]["cus"] = torch.cuda.get_device_properties(0).multi_processor_count
    except Exception:
        pass
    if args.serve_seconds > 0:
        log(f"serving 8, 16, 32 and 64 sessions, {args.serve_seconds} s each ...")
        sweep = serve_sweep(L, scene, cloud, blob, args.serve_seconds)
        line["serving"] = dict(sweep[-1])  # the 64-session workload
        line["serving"]["sweep"] = [{k: r[k] for k in ("sessions", "offered_requests_per_s", "frames_per_s",
                                                       "superseded_fraction", "latency_ms", "superseded_wait_ms",
                                                       "mean_batch", "megapixels_per_s")} for r in sweep]
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample ...")
        line["cpu_baseline"] = cpu_baseline(scene, cams, blob, NL, FS, widths, geo_pre)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
