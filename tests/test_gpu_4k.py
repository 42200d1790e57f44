"""Parity at the shape of the largest configuration: 3840x2160 views, depth
filter with 6 levels and filter_strength 0.5, a 5-level U-Net with widths
32/64/128/256/512, batches of 8 views.  The cloud is the 20M-point multi-room
scene (1 m cells); the 300M-point cloud of that configuration changes how
many points are culled and splatted, not the shapes the kernels see.

Projection and filter are compared on the whole 4K frame bit for bit, the
U-Net on 64x64 windows (corners included) against the float64 oracle, and a
batch of 8 served 4K views against the same views computed alone."""

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

W, H, FOV, NL, FS, CELL = 3840, 2160, 90.0, 6, 0.5, 1.0
WIDTHS = (32, 64, 128, 256, 512)
WINDOWS = [(0, 64, 0, 64), (H - 64, H, W - 64, W), (1000, 1064, 2901, 2965)]


@pytest.fixture(scope="module")
def four_k(lnr, ctx):
    scene = synth.scene_for_config("multiroom", seed=0)
    cloud = lnr.lnr_cloud_load(ctx, scene.xyz, scene.rgb, CELL)
    cam = synth.orbit_path(scene, 120, W, H, FOV)[17]
    key, depth, rgba = R.render(G.partition(scene.xyz, scene.rgb, CELL), cam)
    fd, fr, _ = F.depth_filter(depth.reshape(H, W), rgba.reshape(H, W, 4), NL, FS)
    blob = synth.make_unet_blob(WIDTHS, seed=5)
    net = U.parse_blob(blob)
    refs = [U.forward_crop(net, fd, fr, *w) for w in WINDOWS]
    return {"scene": scene, "cloud": cloud, "cam": cam, "oracle": (key, depth, rgba, fd, fr), "blob": blob,
            "refs": refs}


def test_4k_render_and_six_level_filter_bit_exact(lnr, ctx, four_k):
    import torch
    key, depth, rgba, fd, fr = four_k["oracle"]
    img = render_gpu(lnr, ctx, four_k["cloud"], four_k["cam"])
    assert_images_equal(image_to_host(img), (key, depth, rgba), "4k render")
    lnr.lnr_depth_filter(ctx, img, NL, FS)
    torch.cuda.synchronize()
    _, gd, gr = image_to_host(img)
    assert_images_equal((None, gd, gr), (None, fd, fr), "4k filter")


@pytest.mark.parametrize("prec", UNET_PRECISIONS)
def test_4k_five_level_unet_sampled_windows(lnr, ctx, four_k, prec):
    import torch
    _, _, _, fd, fr = four_k["oracle"]
    net = lnr.lnr_unet_load(ctx, four_k["blob"], prec)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    lnr.lnr_reconstruct(ctx, net, image_from_host(lnr, fd, fr), out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    worst = max(M.max_abs(got[:, a:b, c:d], ref) for (a, b, c, d), ref in zip(WINDOWS, four_k["refs"]))
    check_unet_error(prec, worst, "4k windows")


@pytest.mark.parametrize("prec,graphs", [("LNR_BF16", False), ("LNR_FP16", True)])
def test_4k_batch_of_eight_views_equals_alone(lnr, ctx, four_k, prec, graphs):
    """Eight 4K views in one batch (widths[0] = 32, so the head is fused and
    every view writes its own output), launched directly or as one captured
    graph of the whole batch."""
    import torch
    net = lnr.lnr_unet_load(ctx, four_k["blob"], getattr(lnr, prec))
    srv = lnr.lnr_server_create(ctx, four_k["cloud"], net, max_batch=8, lanes=1, n_levels=NL, filter_strength=FS,
                                use_graphs=graphs, max_width=W, max_height=H)
    sids = [lnr.lnr_server_open_session(srv, W, H) for _ in range(8)]
    cams = [synth.random_walk_path(four_k["scene"], 1, seed=200 + i, width=W, height=H, fov_deg=FOV)[0]
            for i in range(8)]
    for i, sid in enumerate(sids):
        lnr.lnr_server_submit(srv, sid, cams[i], tag=i)
    results = {}
    for _ in range(100000):
        lnr.lnr_server_step(srv)
        for r in lnr.lnr_server_poll(srv):
            assert not r["superseded"]
            o = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
            lnr.copy_from_device(r["rgb"], o)
            results[r["tag"]] = (o.cpu().numpy(), r["batch"])
        if len(results) == 8:
            break
    assert len(results) == 8, "server did not finish"
    assert max(b for _, b in results.values()) == 8, "the eight views were not served as one batch"
    lnr.lnr_server_destroy(srv)
    for i, cam in enumerate(cams):
        img = render_gpu(lnr, ctx, four_k["cloud"], cam)
        lnr.lnr_depth_filter(ctx, img, NL, FS)
        alone = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
        lnr.lnr_reconstruct(ctx, net, img, alone)
        torch.cuda.synchronize()
        assert np.array_equal(results[i][0], alone.cpu().numpy()), f"view {i} differs from its standalone frame"


@pytest.mark.parametrize("frame", [0, 61])
def test_4k_largest_scene_layout_bit_exact(lnr, ctx, frame):
    """The largest configuration's building (80 x 60 x 10 m, 32 rooms, 16
    scans, 2 m cells) at 4M points instead of 300M: projection and the
    6-level filter of a 4K view of its orbit path, bit for bit."""
    import torch
    scene = synth.scene_for_config("huge", seed=0, n_points=4_000_000)
    cloud = lnr.lnr_cloud_load(ctx, scene.xyz, scene.rgb, 2.0)
    cam = synth.orbit_path(scene, 120, W, H, FOV)[frame]
    key, depth, rgba = R.render(G.partition(scene.xyz, scene.rgb, 2.0), cam)
    fd, fr, _ = F.depth_filter(depth.reshape(H, W), rgba.reshape(H, W, 4), NL, FS)
    assert (rgba.reshape(H, W, 4)[..., 3] != 0).mean() > 0.02, "the view sees too little of the scene"
    img = render_gpu(lnr, ctx, cloud, cam)
    assert_images_equal(image_to_host(img), (key, depth, rgba), f"largest-layout render {frame}")
    lnr.lnr_depth_filter(ctx, img, NL, FS)
    torch.cuda.synchronize()
    _, gd, gr = image_to_host(img)
    assert_images_equal((None, gd, gr), (None, fd, fr), f"largest-layout filter {frame}")
    lnr.lnr_cloud_destroy(cloud)


def test_4k_eight_views_in_one_pass(lnr, ctx):
    """The largest configuration's building at 4M points: 8 consecutive 4K
    orbit views projected in one pass (lnr_render_views) equal each view
    rendered alone, and views 0 and 7 equal the oracle, bit for bit."""
    import torch
    scene = synth.scene_for_config("huge", seed=0, n_points=4_000_000)
    cloud = lnr.lnr_cloud_load(ctx, scene.xyz, scene.rgb, 2.0)
    cams = synth.orbit_path(scene, 120, W, H, FOV)[40:48]
    imgs = [lnr.Image(H, W) for _ in cams]
    lnr.lnr_render_views(ctx, cloud, cams, imgs)
    torch.cuda.synchronize()
    g = G.partition(scene.xyz, scene.rgb, 2.0)
    for v, cam in enumerate(cams):
        got = image_to_host(imgs[v])
        assert_images_equal(got, image_to_host(render_gpu(lnr, ctx, cloud, cam)), f"view {v} vs alone")
        if v in (0, 7):
            assert_images_equal(got, R.render(g, cam), f"view {v} vs oracle")
    lnr.lnr_cloud_destroy(cloud)
