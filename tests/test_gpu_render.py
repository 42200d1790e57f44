"""GPU parity of the partition, culling, splat and resolve against the oracle
(bit-exact), through the C ABI."""

import numpy as np
import pytest

import synth
from oracle import grid as G
from oracle import render as R
from tests.gpu_util import assert_images_equal, image_to_host, render_gpu

pytestmark = pytest.mark.gpu


def test_partition_matches_oracle(lnr, room_cloud, room_grid):
    info = lnr.lnr_cloud_info(room_cloud)
    assert info["dims"] == room_grid.dims
    assert np.array_equal(info["origin"], room_grid.lo)
    assert np.array_equal(lnr.lnr_cloud_permutation(room_cloud), room_grid.perm.astype(np.uint32))
    assert np.array_equal(lnr.lnr_cloud_cell_start(room_cloud), room_grid.cell_start.astype(np.uint32))


@pytest.mark.parametrize("seed,n,s", [(0, 1, 0.5), (1, 7, 0.01), (2, 100_000, 0.5), (3, 300_000, 2.0),
                                      (4, 50_000, 0.1)])
def test_partition_random_clouds(lnr, ctx, seed, n, s):
    """Stable order with duplicated points, a grid of millions of mostly empty
    cells (0.1 m cells over a Gaussian cloud of radius ~8 m) and a single point."""
    rng = np.random.default_rng(seed)
    xyz = (rng.standard_normal((n, 3)) * 2).astype(np.float32)
    if n > 20:
        xyz[n // 3:n // 3 + 10] = xyz[:10]
    rgb = rng.integers(0, 256, (n, 3), dtype=np.uint8)
    g = G.partition(xyz, rgb, s)
    cloud = lnr.lnr_cloud_load(ctx, xyz, rgb, s)
    assert lnr.lnr_cloud_info(cloud)["dims"] == g.dims
    assert np.array_equal(lnr.lnr_cloud_permutation(cloud), g.perm.astype(np.uint32))
    assert np.array_equal(lnr.lnr_cloud_cell_start(cloud), g.cell_start.astype(np.uint32))


def test_cloud_load_rejects_bad_input(lnr, ctx):
    rng = np.random.default_rng(0)
    xyz = (rng.standard_normal((1000, 3)) * 2).astype(np.float32)
    rgb = np.zeros((1000, 3), np.uint8)
    for bad_s in (0.003, 0.0, -1.0, float("nan"), float("inf")):  # 0.003 m: more than 2^31 cells
        with pytest.raises(lnr.LnrError) as e:
            lnr.lnr_cloud_load(ctx, xyz, rgb, bad_s)
        assert e.value.status == lnr.LNR_E_INVALID_ARG
    xyz[5, 1] = np.nan
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_cloud_load(ctx, xyz, rgb, 0.5)
    assert e.value.status == lnr.LNR_E_INVALID_ARG


def test_budget_is_enforced(lnr, room_scene):
    small = lnr.lnr_context_create(0, 1 << 20)
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_cloud_load(small, room_scene.xyz, room_scene.rgb, 0.5)
    assert e.value.status == lnr.LNR_E_BUDGET
    assert lnr.lnr_allocated_bytes(small) == 0


@pytest.mark.parametrize("i", range(16))
def test_render_room_bit_exact(lnr, ctx, room_cloud, room_grid, room_cams, i):
    cam = room_cams[i]
    img = render_gpu(lnr, ctx, room_cloud, cam)
    vis_gpu, proc_gpu, flags = lnr.lnr_render_stats(ctx, room_grid.n_cells)
    key, depth, rgba = R.render(room_grid, cam)
    assert_images_equal(image_to_host(img), (key, depth, rgba), f"frame {i}")
    vis = G.cull(room_grid, cam.P, cam.width, cam.height, cam.z_near, cam.z_far)
    assert np.array_equal(flags, vis)
    assert vis_gpu == int(vis.sum())
    assert proc_gpu == R.processed_points(room_grid, vis)


def test_culled_render_equals_unculled(lnr, ctx, room_cloud, room_cams):
    for cam in room_cams[:6]:
        a = image_to_host(render_gpu(lnr, ctx, room_cloud, cam))
        b = image_to_host(render_gpu(lnr, ctx, room_cloud, cam, flags=lnr.LNR_RENDER_NO_CULL))
        assert_images_equal(a, b, "cull vs no cull")
        _, proc_all, _ = lnr.lnr_render_stats(ctx)
        assert proc_all == 200_000


def test_render_grazing_cameras(lnr, ctx, room_cloud, room_grid):
    """Cameras inside the cloud with near planes and image borders cutting
    through it, narrow and wide fields of view, odd image sizes."""
    rng = np.random.default_rng(11)
    xyz = room_grid
    for t in range(24):
        j, k = rng.integers(0, len(room_grid.xs), 2)
        eye = np.array([room_grid.xs[j], room_grid.ys[j], room_grid.zs[j]], np.float64) + rng.normal(0, 0.2, 3)
        tgt = np.array([room_grid.xs[k], room_grid.ys[k], room_grid.zs[k]], np.float64)
        if np.linalg.norm(tgt - eye) < 0.3:
            continue
        W, H = int(rng.integers(1, 200)), int(rng.integers(1, 200))
        cam = synth.look_at(eye, tgt, W, H, float(rng.uniform(10, 150)), float(rng.choice([0.1, 1.0, 3.0])),
                            float(rng.choice([4.0, 1000.0])))
        img = render_gpu(lnr, ctx, room_cloud, cam)
        assert_images_equal(image_to_host(img), R.render(room_grid, cam), f"grazing {t}")


def test_render_empty_view_and_tiny_image(lnr, ctx, room_cloud, room_grid):
    cam = synth.look_at([-5, 4, 1.5], [-10, 4, 1.5], 64, 48, 70.0)  # outside, looking away
    img = render_gpu(lnr, ctx, room_cloud, cam)
    k, d, r = image_to_host(img)
    assert np.all(k == np.uint64(lnr.EMPTY_KEY)) and not d.any() and not r.any()
    vis, proc, _ = lnr.lnr_render_stats(ctx)
    assert vis == 0 and proc == 0
    cam = synth.look_at([5, 4, 1.5], [9, 4, 1.5], 1, 1, 60.0)
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, room_cloud, cam)), R.render(room_grid, cam), "1x1")


def test_render_ties_and_duplicates(lnr, ctx):
    """Many points at the same depth in one pixel and exact duplicates: the
    lowest sorted index wins, as in the oracle."""
    rng = np.random.default_rng(3)
    base = np.float32([[2.0, 0.01, 0.01], [2.0, 0.02, 0.01], [2.0, 0.01, 0.02]])
    xyz = np.concatenate([np.repeat(base, 200, axis=0), rng.uniform(-1, 3, (5000, 3)).astype(np.float32)])
    rgb = rng.integers(0, 256, xyz.shape, dtype=np.uint8)
    g = G.partition(xyz, rgb, 0.25)
    cloud = lnr.lnr_cloud_load(ctx, xyz, rgb, 0.25)
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 16, 16, 90.0)
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, cloud, cam)), R.render(g, cam), "ties")


def test_render_large_image(lnr, ctx, room_cloud, room_grid):
    cam = synth.look_at([5, 4, 1.5], [9, 2, 1.2], 4096, 3072, 100.0)
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, room_cloud, cam)), R.render(room_grid, cam), "4k")


def test_render_rejects_bad_arguments(lnr, ctx, room_cloud, room_cams):
    import torch
    cam = room_cams[0]
    img = lnr.Image(cam.height, cam.width + 1)
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_render(ctx, room_cloud, cam, img)
    assert e.value.status == lnr.LNR_E_INVALID_ARG
    c = lnr.camera_struct(cam)
    c.z_near = 0.0
    with pytest.raises(lnr.LnrError):
        lnr.lnr_render(ctx, room_cloud, c, lnr.Image(cam.height, cam.width))
    torch.cuda.synchronize()


@pytest.mark.parametrize("eps", [0.0, 0.01, 0.05])
def test_soft_zbuffer_bit_exact(lnr, ctx, room_cloud, room_grid, room_cams, eps):
    """The paper's soft z-buffer: colour = rounded mean over points within
    (1 + eps) of the nearest depth; key and depth stay the nearest point's."""
    import torch
    g = room_grid
    for i, cam in enumerate(room_cams[:6]):
        img = lnr.Image(cam.height, cam.width)
        lnr.lnr_render_soft(ctx, room_cloud, cam, img, eps)
        torch.cuda.synchronize()
        key, depth, _ = R.render(g, cam)
        rgba = R.soft_colors(g.xs, g.ys, g.zs, g.rgb, cam.P, cam.width, cam.height, cam.z_near, cam.z_far, key, eps)
        assert_images_equal(image_to_host(img), (key, depth, rgba), f"soft eps={eps} frame {i}")


def test_soft_zbuffer_rejects_bad_eps(lnr, ctx, room_cloud, room_cams):
    cam = room_cams[0]
    for eps in (-0.1, float("nan"), float("inf")):
        with pytest.raises(lnr.LnrError) as e:
            lnr.lnr_render_soft(ctx, room_cloud, cam, lnr.Image(cam.height, cam.width), eps)
        assert e.value.status == lnr.LNR_E_INVALID_ARG


def test_objects_outlive_a_destroyed_context(lnr, ctx, room_scene, room_grid, room_cams):
    """Destroying a context before its cloud and network (as a garbage
    collector may) keeps them usable and leaves no error behind for later
    calls: the context is freed with its last object."""
    import torch
    c1 = lnr.lnr_context_create(0)
    cloud = lnr.lnr_cloud_load(c1, room_scene.xyz, room_scene.rgb, 0.5)
    net = lnr.lnr_unet_load(c1, synth.make_unet_blob((16, 32), seed=0), lnr.LNR_BF16)
    lnr.lnr_context_destroy(c1)
    cam = room_cams[3]
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, cloud, cam)), R.render(room_grid, cam), "after destroy")
    out = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device="cuda")
    lnr.lnr_reconstruct(ctx, net, render_gpu(lnr, ctx, cloud, cam), out)
    torch.cuda.synchronize()
    lnr.lnr_unet_destroy(net)
    lnr.lnr_cloud_destroy(cloud)    # frees the context too
    fresh = lnr.lnr_cloud_load(ctx, room_scene.xyz, room_scene.rgb, 0.5)
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, fresh, cam)), R.render(room_grid, cam), "fresh cloud")


@pytest.mark.parametrize("i", [0, 5, 11])
def test_counting_render_is_bit_exact_and_counts_plausibly(lnr, ctx, room_cloud, room_grid, room_cams, i):
    """The atomic-counting projection writes the same image; its count of
    z-buffer atomics lies between the filled pixels (the first point on an
    empty pixel always issues one) and the processed points (at most one per
    point).  The count depends on the order points arrive in, so only these
    bounds are checked."""
    cam = room_cams[i]
    plain = image_to_host(render_gpu(lnr, ctx, room_cloud, cam))
    img = render_gpu(lnr, ctx, room_cloud, cam, flags=lnr.LNR_RENDER_COUNT_ATOMICS)
    counted = image_to_host(img)
    assert_images_equal(counted, plain, f"counting render {i}")
    assert_images_equal(counted, R.render(room_grid, cam), f"counting render {i} vs oracle")
    n = lnr.lnr_render_atomic_count(ctx)
    _, processed, _ = lnr.lnr_render_stats(ctx)
    filled = int((counted[2].reshape(-1, 4)[:, 3] != 0).sum())
    assert filled > 0
    assert filled <= n <= processed
    render_gpu(lnr, ctx, room_cloud, cam)
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_render_atomic_count(ctx)
    assert e.value.status == lnr.LNR_E_INVALID_ARG


def test_tiled_splat_equals_atomic_splat(lnr, ctx, room_cloud, room_grid, room_cams):
    """The default screen-tiled splat (points binned per 32 x 32 tile, each
    tile's z-buffer on chip) and the atomic one (global z-buffer lowered with
    atomicMin) give the same key, depth and rgba: on the room frames and on
    grazing cameras with odd image sizes (partial tiles at the borders)."""
    rng = np.random.default_rng(5)
    cams = list(room_cams[:8])
    while len(cams) < 20:
        j, k = rng.integers(0, len(room_grid.xs), 2)
        eye = np.array([room_grid.xs[j], room_grid.ys[j], room_grid.zs[j]], np.float64) + rng.normal(0, 0.3, 3)
        tgt = np.array([room_grid.xs[k], room_grid.ys[k], room_grid.zs[k]], np.float64)
        if np.linalg.norm(tgt - eye) < 0.3:
            continue
        cams.append(synth.look_at(eye, tgt, int(rng.integers(1, 300)), int(rng.integers(1, 300)),
                                  float(rng.uniform(20, 160))))
    for i, cam in enumerate(cams):
        a = image_to_host(render_gpu(lnr, ctx, room_cloud, cam))
        b = image_to_host(render_gpu(lnr, ctx, room_cloud, cam, flags=lnr.LNR_RENDER_ATOMIC_SPLAT))
        assert_images_equal(a, b, f"tiled vs atomic, camera {i} ({cam.width}x{cam.height})")


def _identity_camera(W, H):
    """(u, v, w) = (x, y, z): the pixel of a point is (floor(x / z), floor(y / z))."""
    return synth.Camera(P=np.float32([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0]), width=W, height=H)


def _check_both_splats(lnr, ctx, xyz, rgb, cell, cam, what):
    g = G.partition(xyz, rgb, cell)
    cloud = lnr.lnr_cloud_load(ctx, xyz, rgb, cell)
    want = R.render(g, cam)
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, cloud, cam)), want, f"{what} tiled")
    assert_images_equal(image_to_host(render_gpu(lnr, ctx, cloud, cam, flags=lnr.LNR_RENDER_ATOMIC_SPLAT)), want,
                        f"{what} atomic")
    return g, want


@pytest.mark.parametrize("bw,bh", [(64, 64), (65, 64), (1, 1), (4096, 1), (1, 4097), (37, 19)])
def test_splat_work_item_rectangle_limits(lnr, ctx, bw, bh):
    """One work item of 4096 points whose pixels fill a bw x bh rectangle: at
    most 4096 pixels keep only the nearest point per pixel on chip before
    binning, larger ones bin every point.  Half the points lie at depth 1 and
    half at depth 2 behind them, with many exact depth ties per pixel (the
    lowest index must win)."""
    rng = np.random.default_rng(bw * 7 + bh)
    n = 4096
    ux = rng.integers(0, bw, n) + 10.25
    vy = rng.integers(0, bh, n) + 20.5
    w = np.where(np.arange(n) % 2 == 0, 1.0, 2.0)
    xyz = np.stack([ux * w, vy * w, w], axis=1).astype(np.float32)
    rgb = rng.integers(0, 256, (n, 3), dtype=np.uint8)
    g, want = _check_both_splats(lnr, ctx, xyz, rgb, 1e4, _identity_camera(bw + 20, bh + 30), f"{bw}x{bh}")
    assert g.n_cells == 1
    assert int((want[2].reshape(-1, 4)[:, 3] != 0).sum()) == len(set(zip(ux.tolist(), vy.tolist())))


@pytest.mark.parametrize("W,H", [(2048, 2048), (3000, 3000), (4000, 1000)])
def test_tiled_splat_work_item_spanning_many_tiles(lnr, ctx, W, H):
    """One cell whose points spread over the whole of a large image: the work
    item touches more tiles (up to 94 x 94) than one binning pass addresses
    (4096), so it is binned in several rounds of tile rows."""
    rng = np.random.default_rng(W + H)
    n = 4000
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    xyz = (d * rng.uniform(1.0, 3.0, (n, 1))).astype(np.float32)
    xyz[:50] = xyz[50:100]  # duplicates: ties go to the lowest index
    rgb = rng.integers(0, 256, (n, 3), dtype=np.uint8)
    cam = synth.look_at([0, 0, 0], [1, 0.1, 0.05], W, H, 170.0)
    g, want = _check_both_splats(lnr, ctx, xyz, rgb, 10.0, cam, f"{W}x{H} single cell")
    assert g.n_cells == 1
    assert int((want[2].reshape(-1, 4)[:, 3] != 0).sum()) > 500


def test_tiled_splat_busy_tiles_split_into_units(lnr, ctx):
    """About 2,300 work items over four 32 x 32 tiles: each of those tiles has
    far more segments than one unit of the tile kernel takes (32), so its
    units merge through the key buffer; the rest of the image is empty
    tiles.  Many points share a pixel, at different and at equal depths."""
    rng = np.random.default_rng(17)
    n = 100_000
    u = rng.uniform(0, 64, n)
    v = rng.uniform(0, 64, n)
    z = rng.choice(np.float32([2.0, 2.5, 3.0]), n) + rng.integers(0, 2, n) * rng.uniform(0, 0.5, n)
    xyz = np.stack([u * z, v * z, z], axis=1).astype(np.float32)
    rgb = rng.integers(0, 256, (n, 3), dtype=np.uint8)
    g, want = _check_both_splats(lnr, ctx, xyz, rgb, 4.0, _identity_camera(100, 70), "busy tiles")
    assert g.n_cells > 1000
    filled = want[2].reshape(70, 100, 4)[..., 3] != 0
    assert filled[:64, :64].mean() > 0.99 and not filled[:, 64:].any()


@pytest.mark.parametrize("pattern", [0, 1])
def test_atomic_min_probe(lnr, ctx, pattern):
    """The throughput probe runs whole blocks of 256 x 64 operations and
    returns a positive rate; it frees its buffer and rejects bad arguments."""
    before = lnr.lnr_allocated_bytes(ctx)
    rate, done = lnr.lnr_measure_atomic_min(ctx, 1920 * 1080, pattern, 1 << 22)
    assert done == 1 << 22
    assert 1e8 < rate < 1e14
    rate2, done2 = lnr.lnr_measure_atomic_min(ctx, 7, pattern, 1)
    assert done2 == 256 * 64 and rate2 > 0
    assert lnr.lnr_allocated_bytes(ctx) == before
    for bad in [dict(n_slots=0), dict(n_slots=1 << 32), dict(pattern=2), dict(n_ops=0)]:
        kw = dict(n_slots=1024, pattern=pattern, n_ops=1024)
        kw.update(bad)
        with pytest.raises(lnr.LnrError) as e:
            lnr.lnr_measure_atomic_min(ctx, **kw)
        assert e.value.status == lnr.LNR_E_INVALID_ARG
