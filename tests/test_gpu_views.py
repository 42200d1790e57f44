"""Several views in one pass over the cloud (lnr_render_views): every view's
key, depth and rgba equal the oracle's render of that camera alone, bit for
bit, and equal lnr_render's; culling, the per-view on-chip z-buffer and the
passes of up to 8 views change nothing in the images.  Through the C ABI."""

import numpy as np
import pytest

import synth
from oracle import grid as G
from oracle import render as R
from tests.gpu_util import assert_images_equal, image_to_host, render_gpu

pytestmark = pytest.mark.gpu


def _render_views(lnr, ctx, cloud, cams, flags=0):
    import torch
    imgs = [lnr.Image(c.height, c.width) for c in cams]
    lnr.lnr_render_views(ctx, cloud, cams, imgs, flags)
    torch.cuda.synchronize()
    return imgs


def _grazing_cams(room_grid, n, seed):
    rng = np.random.default_rng(seed)
    cams = []
    while len(cams) < n:
        j, k = rng.integers(0, len(room_grid.xs), 2)
        eye = np.array([room_grid.xs[j], room_grid.ys[j], room_grid.zs[j]], np.float64) + rng.normal(0, 0.3, 3)
        tgt = np.array([room_grid.xs[k], room_grid.ys[k], room_grid.zs[k]], np.float64)
        if np.linalg.norm(tgt - eye) < 0.3:
            continue
        cams.append(synth.look_at(eye, tgt, int(rng.integers(1, 300)), int(rng.integers(1, 300)),
                                  float(rng.uniform(20, 160)), float(rng.choice([0.1, 1.0])),
                                  float(rng.choice([4.0, 1000.0]))))
    return cams


def test_views_equal_oracle_over_three_passes(lnr, ctx, room_cloud, room_grid, room_cams):
    """16 orbit frames and 3 grazing cameras of odd sizes: 19 views, i.e.
    passes of 8, 8 and 3.  The statistics describe the last pass: the cells
    visible in any of its views and their points, each read once."""
    cams = list(room_cams[:16]) + _grazing_cams(room_grid, 3, seed=21)
    imgs = _render_views(lnr, ctx, room_cloud, cams)
    vis_gpu, proc_gpu, flags = lnr.lnr_render_stats(ctx, room_grid.n_cells)
    for v, (cam, img) in enumerate(zip(cams, imgs)):
        assert_images_equal(image_to_host(img), R.render(room_grid, cam), f"view {v} ({cam.width}x{cam.height})")
    union = np.zeros(room_grid.n_cells, bool)
    for cam in cams[16:]:
        union |= G.cull(room_grid, cam.P, cam.width, cam.height, cam.z_near, cam.z_far).astype(bool)
    assert np.array_equal(flags.astype(bool), union)
    assert vis_gpu == int(union.sum())
    assert proc_gpu == R.processed_points(room_grid, union)
    assert proc_gpu <= sum(R.processed_points(room_grid, G.cull(room_grid, c.P, c.width, c.height, c.z_near,
                                                                c.z_far)) for c in cams[16:])


def test_views_equal_single_renders(lnr, ctx, room_cloud, room_grid, room_cams):
    """One view, and 8 views of a batch in one pass, against lnr_render of
    each camera alone (tiled and atomic splats) and against the unculled
    multi-view render."""
    cams = [room_cams[i] for i in (0, 1, 2, 3, 6, 9, 12, 15)]
    one = _render_views(lnr, ctx, room_cloud, cams[:1])
    assert_images_equal(image_to_host(one[0]), image_to_host(render_gpu(lnr, ctx, room_cloud, cams[0])), "1 view")
    culled = _render_views(lnr, ctx, room_cloud, cams)
    unculled = _render_views(lnr, ctx, room_cloud, cams, flags=lnr.LNR_RENDER_NO_CULL)
    for v, cam in enumerate(cams):
        a = image_to_host(culled[v])
        assert_images_equal(a, image_to_host(render_gpu(lnr, ctx, room_cloud, cam)), f"view {v} vs tiled")
        assert_images_equal(a, image_to_host(render_gpu(lnr, ctx, room_cloud, cam,
                                                        flags=lnr.LNR_RENDER_ATOMIC_SPLAT)), f"view {v} vs atomic")
        assert_images_equal(a, image_to_host(unculled[v]), f"view {v} culled vs unculled")


def test_views_repeated_camera_and_empty_view(lnr, ctx, room_cloud, room_grid, room_cams):
    """The same camera in several views fills each image alike; a view that
    sees nothing comes out empty while its pass-mates draw."""
    away = synth.look_at([-5, 4, 1.5], [-10, 4, 1.5], 64, 48, 70.0)
    cams = [room_cams[7], away, room_cams[7], room_cams[7]]
    imgs = _render_views(lnr, ctx, room_cloud, cams)
    want = R.render(room_grid, room_cams[7])
    for v in (0, 2, 3):
        assert_images_equal(image_to_host(imgs[v]), want, f"repeated view {v}")
    k, d, r = image_to_host(imgs[1])
    assert np.all(k == np.uint64(lnr.EMPTY_KEY)) and not d.any() and not r.any()


def _identity_like(W, H, sx, tx):
    """(u, v, w) = (sx x + tx w, y, z): pixel (floor(sx x / z + tx), floor(y / z))."""
    return synth.Camera(P=np.float32([sx, 0, tx, 0, 0, 1, 0, 0, 0, 0, 1, 0]), width=W, height=H)


def test_views_dedup_and_direct_paths_in_one_pass(lnr, ctx):
    """One work item of 4096 points over a 64 x 64 pixel square, seen by views
    that stretch it (128 x 64: more than the 4096 pixels of the on-chip
    z-buffer, so points go one by one), shift it half out of the image, or
    keep it: each view takes its own path, and every image equals the
    oracle's.  Half the points lie behind the others, with exact depth ties."""
    rng = np.random.default_rng(9)
    n = 4096
    ux = rng.integers(0, 64, n) + 0.25
    vy = rng.integers(0, 64, n) + 0.5
    w = np.where(np.arange(n) % 2 == 0, 1.0, 2.0)
    xyz = np.stack([ux * w, vy * w, w], axis=1).astype(np.float32)
    rgb = rng.integers(0, 256, (n, 3), dtype=np.uint8)
    g = G.partition(xyz, rgb, 1e4)
    assert g.n_cells == 1
    cloud = lnr.lnr_cloud_load(ctx, xyz, rgb, 1e4)
    cams = [_identity_like(80, 70, 1.0, 0.0), _identity_like(140, 70, 2.0, 0.0), _identity_like(80, 70, 1.0, -32.0),
            _identity_like(64, 64, 1.0, 0.0), _identity_like(200, 70, 2.0, 5.0)]
    imgs = _render_views(lnr, ctx, cloud, cams)
    for v, cam in enumerate(cams):
        assert_images_equal(image_to_host(imgs[v]), R.render(g, cam), f"view {v}")


def test_views_reject_bad_arguments_before_drawing(lnr, ctx, room_cloud, room_cams):
    import torch
    cams = list(room_cams[:3])

    def sentinel(c):
        img = lnr.Image(c.height, c.width)
        img.key.fill_(0x5A5A5A5A5A5A5A5A)
        img.depth.fill_(-3.25)
        return img

    def untouched(imgs):
        torch.cuda.synchronize()
        return all(bool((i.key == 0x5A5A5A5A5A5A5A5A).all()) and bool((i.depth == -3.25).all()) for i in imgs)

    imgs = [sentinel(c) for c in cams]
    bad_size = [imgs[0], imgs[1], lnr.Image(cams[2].height + 1, cams[2].width)]
    # a third view whose depth plane is the second view's
    shared_depth = lnr.Image.from_tensors(imgs[1].depth, lnr.Image(cams[2].height, cams[2].width).rgba,
                                          lnr.Image(cams[2].height, cams[2].width).key)
    for args, what in [((cams, bad_size, 0), "size of the last view"),
                       ((cams, [imgs[0], imgs[1], imgs[0]], 0), "shared key buffer"),
                       ((cams, [imgs[0], imgs[1], shared_depth], 0), "shared depth buffer"),
                       ((cams, imgs, lnr.LNR_RENDER_ATOMIC_SPLAT), "flag"),
                       ((cams[:0], imgs[:0], 0), "no view")]:
        with pytest.raises(lnr.LnrError) as e:
            lnr.lnr_render_views(ctx, room_cloud, *args)
        assert e.value.status == lnr.LNR_E_INVALID_ARG, what
        assert untouched(imgs), what
    c = lnr.camera_struct(cams[1])
    c.z_near = 0.0
    with pytest.raises(lnr.LnrError):
        lnr.lnr_render_views(ctx, room_cloud, [cams[0], c, cams[2]], imgs)
    assert untouched(imgs)
