"""Parity at the full frame-rate workload, in the launch configuration the
bench times: 20M points of the seeded multi-room scene in 1 m cells, the
1920x1080 orbit path (90 degree fov), depth filter with 5 levels and
filter_strength 0.5, U-Net widths 32/64/128/256.

Projection and filter are compared on whole frames, bit for bit.  The U-Net is
compared on six 64x64 windows that the float64 oracle computes one by one on
a crop grown by the receptive margin (corners, so the ragged tile tails of
every level are covered; two windows across the tile seams of every level),
with the bounds of the small-size tests.  Batched serving at this size must give each frame exactly what it
gives alone."""

import numpy as np
import pytest

import synth
from oracle import depth_filter as F
from oracle import grid as G
from oracle import metrics as M
from oracle import render as R
from oracle import unet as U
from tests.gpu_util import FP32, UNET_PRECISIONS, check_unet_error, assert_images_equal, image_from_host, image_to_host, render_gpu

pytestmark = pytest.mark.gpu

W, H, FOV, NL, FS, CELL = 1920, 1080, 90.0, 5, 0.5, 1.0
WIDTHS = (32, 64, 128, 256)
FRAMES = (0, 30, 60, 90)
UNET_FRAMES = (0, 60)


def _windows(frame):
    """Corners (the ragged tile tails of every level), the centre, a random
    window, and two windows that straddle the convolution tile seams of every
    level: a workgroup tile is 8 rows x 32 columns of level-l pixels, i.e.
    8 * 2^l by 32 * 2^l full-resolution pixels, so rows 128 and 512 and
    columns 256 and 1024 are seams at levels 0-3 (and 0-4 for the rows)."""
    rng = np.random.default_rng(1000 + frame)
    y, x = int(rng.integers(0, H - 64)), int(rng.integers(0, W - 64))
    return [(0, 64, 0, 64), (H - 64, H, W - 64, W), (H // 2 - 32, H // 2 + 32, W // 2 - 32, W // 2 + 32),
            (y, y + 64, x, x + 64), (96, 160, 224, 288), (480, 544, 992, 1056)]


@pytest.fixture(scope="module")
def full(lnr, ctx):
    scene = synth.scene_for_config("multiroom", seed=0)
    grid = G.partition(scene.xyz, scene.rgb, CELL)
    cloud = lnr.lnr_cloud_load(ctx, scene.xyz, scene.rgb, CELL)
    cams = synth.orbit_path(scene, 120, W, H, FOV)
    blob = synth.make_unet_blob(WIDTHS, seed=0)
    filtered = {}
    for f in FRAMES:
        key, depth, rgba = R.render(grid, cams[f])
        fd, fr, _ = F.depth_filter(depth.reshape(H, W), rgba.reshape(H, W, 4), NL, FS)
        filtered[f] = (key, depth, rgba, fd, fr)
    return {"scene": scene, "cloud": cloud, "cams": cams, "blob": blob, "oracle": filtered, "refs": {}}


def _refs(full, f):
    if f not in full["refs"]:
        net = U.parse_blob(full["blob"])
        _, _, _, fd, fr = full["oracle"][f]
        full["refs"][f] = [U.forward_crop(net, fd, fr, *w) for w in _windows(f)]
    return full["refs"][f]


def test_fullsize_render_and_filter_bit_exact(lnr, ctx, full):
    for f in FRAMES:
        print(f"frame {f}", flush=True)
        key, depth, rgba, fd, fr = full["oracle"][f]
        img = render_gpu(lnr, ctx, full["cloud"], full["cams"][f])
        assert_images_equal(image_to_host(img), (key, depth, rgba), f"render frame {f}")
        lnr.lnr_depth_filter(ctx, img, NL, FS)
        import torch
        torch.cuda.synchronize()
        _, gd, gr = image_to_host(img)
        assert_images_equal((None, gd, gr), (None, fd, fr), f"filter frame {f}")


@pytest.mark.parametrize("prec", UNET_PRECISIONS)
def test_fullsize_unet_sampled_windows(lnr, ctx, full, prec):
    import torch
    net = lnr.lnr_unet_load(ctx, full["blob"], prec)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    worst = 0.0
    for f in UNET_FRAMES:
        print(f"prec {prec} frame {f}", flush=True)
        _, _, _, fd, fr = full["oracle"][f]
        lnr.lnr_reconstruct(ctx, net, image_from_host(lnr, fd, fr), out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().astype(np.float64)
        for (a, b, c, d), ref in zip(_windows(f), _refs(full, f)):
            worst = max(worst, M.max_abs(got[:, a:b, c:d], ref))
    check_unet_error(prec, worst, "1080p windows")


@pytest.mark.parametrize("prec", [0, 1, 4])
def test_fullsize_batched_serving_equals_alone(lnr, ctx, full, prec):
    import torch
    net = lnr.lnr_unet_load(ctx, full["blob"], prec)
    srv = lnr.lnr_server_create(ctx, full["cloud"], net, max_batch=4, lanes=1, n_levels=NL, filter_strength=FS,
                                use_graphs=True, max_width=W, max_height=H)
    sizes = [(W, H), (W, H), (1280, 720), (W, H)]
    sids = [lnr.lnr_server_open_session(srv, w, h) for (w, h) in sizes]
    cams = [synth.random_walk_path(full["scene"], 2, seed=50 + i, width=w, height=h, fov_deg=FOV)
            for i, (w, h) in enumerate(sizes)]
    results = {}
    for f in range(2):
        for i, sid in enumerate(sids):
            lnr.lnr_server_submit(srv, sid, cams[i][f], tag=f * 10 + i)
        for _ in range(100000):
            lnr.lnr_server_step(srv)
            for r in lnr.lnr_server_poll(srv):
                assert not r["superseded"]
                o = torch.empty((3, r["height"], r["width"]), dtype=torch.float32, device="cuda")
                lnr.copy_from_device(r["rgb"], o)
                results[r["tag"]] = (o.cpu().numpy(), r["batch"])
            if len(results) == (f + 1) * len(sids):
                break
        assert len(results) == (f + 1) * len(sids), "server did not finish"
    assert max(b for _, b in results.values()) >= 3, "no 1080p batch of three was formed"
    lnr.lnr_server_destroy(srv)
    for f in range(2):
        for i in range(len(sizes)):
            cam = cams[i][f]
            img = render_gpu(lnr, ctx, full["cloud"], cam)
            lnr.lnr_depth_filter(ctx, img, NL, FS)
            alone = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device="cuda")
            lnr.lnr_reconstruct(ctx, net, img, alone)
            torch.cuda.synchronize()
            assert np.array_equal(results[f * 10 + i][0], alone.cpu().numpy()), \
                f"session {i} frame {f} differs from its standalone frame"
