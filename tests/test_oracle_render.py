"""Pins of the oracle's point projection, z-buffer and resolve (CPU only)."""

import numpy as np
import pytest

import synth
from oracle import grid as G
from oracle import render as R

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def _project64(xyz, cam):
    P = cam.P.astype(np.float64).reshape(3, 4)
    h = np.concatenate([xyz.astype(np.float64), np.ones((len(xyz), 1))], 1) @ P.T
    return h[:, 0] / h[:, 2], h[:, 1] / h[:, 2], h[:, 2]


def _cloud_off_borders(rng, cam, n, zrange=(0.5, 20.0), dup=0):
    """Points whose float64 projections sit >= 0.05 px from every pixel border."""
    P = cam.P.astype(np.float64).reshape(3, 4)
    W, H = cam.width, cam.height
    u = rng.integers(-2, W + 2, n) + rng.uniform(0.05, 0.95, n)
    v = rng.integers(-2, H + 2, n) + rng.uniform(0.05, 0.95, n)
    z = rng.uniform(*zrange, n)
    pts = []
    for ui, vi, zi in zip(u, v, z):
        A = np.array([P[0, :3] - ui * P[2, :3], P[1, :3] - vi * P[2, :3], P[2, :3]])
        rhs = np.array([ui * P[2, 3] - P[0, 3], vi * P[2, 3] - P[1, 3], zi - P[2, 3]])
        pts.append(np.linalg.solve(A, rhs))
    xyz = np.array(pts, dtype=np.float32)
    if dup:
        xyz = np.concatenate([xyz, xyz[:dup]])
    return xyz


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_splat_equals_per_pixel_exhaustive_search(seed):
    """For every pixel, scan all points and keep the nearest one landing on it
    (float64 projection; points are kept away from pixel borders so the float32
    and float64 pixels agree), ties to the lowest index."""
    rng = np.random.default_rng(seed)
    cam = synth.look_at(rng.normal(0, 1, 3), rng.normal(0, 1, 3) + [10, 0, 0], 32, 24, 60.0, 0.1, 1000.0)
    xyz = _cloud_off_borders(rng, cam, 1500, dup=40)
    u, v, w = _project64(xyz, cam)
    key = R.splat(xyz[:, 0], xyz[:, 1], xyz[:, 2], cam.P, 32, 24, cam.z_near, cam.z_far)
    wf = (w.astype(np.float32))
    for py in range(24):
        for px in range(32):
            best = None
            for j in range(len(xyz)):
                if not (cam.z_near <= w[j] <= cam.z_far):
                    continue
                if int(np.floor(u[j])) == px and int(np.floor(v[j])) == py:
                    cand = (float(wf[j]), j)
                    if best is None or cand < best:
                        best = cand
            got = key[py * 32 + px]
            if best is None:
                assert got == EMPTY
            else:
                assert int(got & np.uint64(0xFFFFFFFF)) == best[1]
                depth = np.uint32(int(got) >> 32).view(np.float32)
                assert abs(float(depth) - w[best[1]]) <= 1e-6 * w[best[1]]


def test_single_point_closed_form():
    # camera at the origin looking down +x: a point on the axis lands on the principal point
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 64, 48, 90.0)
    key = R.splat(np.float32([3.0]), np.float32([0.0]), np.float32([0.0]), cam.P, 64, 48, 0.1, 1000.0)
    (idx,) = np.nonzero(key != EMPTY)
    assert idx.tolist() == [24 * 64 + 32]
    assert np.uint32(int(key[idx[0]]) >> 32).view(np.float32) == np.float32(3.0)
    # f = 32 px for a 90 degree horizontal fov at W = 64: a point at lateral offset
    # -1.5 m (world -y is image right) at depth 3 is 16 px right of centre
    key = R.splat(np.float32([3.0]), np.float32([-1.5]), np.float32([0.0]), cam.P, 64, 48, 0.1, 1000.0)
    (idx,) = np.nonzero(key != EMPTY)
    assert idx.tolist() == [24 * 64 + 48]


def test_ties_go_to_the_lowest_index():
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 16, 16, 90.0)
    # three points at the same depth inside one pixel, and a duplicate of each
    pts = np.float32([[2.0, 0.01, 0.01], [2.0, 0.02, 0.01], [2.0, 0.01, 0.02]])
    xyz = np.concatenate([pts, pts])
    key = R.splat(xyz[:, 0], xyz[:, 1], xyz[:, 2], cam.P, 16, 16, 0.1, 1000.0)
    hits = key[key != EMPTY]
    assert len(hits) == 1 and int(hits[0] & np.uint64(0xFFFFFFFF)) == 0
    # nearer point wins over lower index
    xyz2 = np.concatenate([pts, np.float32([[1.5, 0.0075, 0.0075]])])
    key2 = R.splat(xyz2[:, 0], xyz2[:, 1], xyz2[:, 2], cam.P, 16, 16, 0.1, 1000.0)
    hits = key2[key2 != EMPTY]
    assert len(hits) == 1 and int(hits[0] & np.uint64(0xFFFFFFFF)) == 3


def test_image_border_is_half_open():
    # f = 32 at W = 64, 90 degrees: lateral offset -+2 m at depth 2 gives u = 64 and u = 0 exactly
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 64, 48, 90.0)
    xyz = np.float32([[2, -2, 0], [2, 2, 0], [2, 0, -1.5], [2, 0, 1.5]])
    valid, pix, _ = R.project(xyz[:, 0], xyz[:, 1], xyz[:, 2], cam.P, 64, 48, 0.1, 1000.0)
    # u = 64 is outside, u = 0 inside; v = 48 (z = -1.5 is image bottom) outside, v = 0 inside
    assert valid.tolist() == [False, True, False, True]
    assert pix[1] == 24 * 64 + 0 and pix[3] == 0 * 64 + 32


def test_clipping_near_far_and_behind():
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 16, 16, 90.0, 1.0, 10.0)
    xyz = np.float32([[-2, 0, 0], [0.5, 0, 0], [1.0, 0, 0], [10.0, 0, 0], [10.5, 0, 0], [5, 100, 0]])
    valid, _, _ = R.project(xyz[:, 0], xyz[:, 1], xyz[:, 2], cam.P, 16, 16, 1.0, 10.0)
    assert valid.tolist() == [False, False, True, True, False, False]


def test_resolve_definition():
    rgb = np.array([[10, 20, 30], [40, 50, 60]], np.uint8)
    k = np.array([EMPTY, (np.uint64(np.float32(2.5).view(np.uint32)) << np.uint64(32)) | np.uint64(1)],
                 dtype=np.uint64)
    depth, rgba = R.resolve(k, rgb)
    assert depth.tolist() == [0.0, 2.5]
    assert rgba.tolist() == [[0, 0, 0, 0], [40, 50, 60, 1]]


def test_camera_at_scanner_sees_first_hits(room_scene):
    """From the scanner position every visible point is a first hit, so the
    nearest depth along each pixel's ray equals the rendered one.  Checked
    statistically: the rendered depth of a pixel is never larger than the depth of
    any point of the cloud that projects to it (definition of a z-buffer)."""
    g = G.partition(room_scene.xyz, room_scene.rgb, 0.5)
    cam = synth.look_at([5, 4, 1.5], [9, 2, 1.0], 96, 96, 80.0)
    key, depth, rgba = R.render(g, cam)
    valid, pix, k = R.project(g.xs, g.ys, g.zs, cam.P, 96, 96, cam.z_near, cam.z_far)
    wbits = (k[valid] >> np.uint64(32)).astype(np.uint32).view(np.float32)
    assert np.all(depth[pix[valid]] <= wbits)
    assert np.all(rgba[pix[valid], 3] == 1)


def test_soft_zbuffer_closed_forms():
    """Two points in one pixel at depths 2.0 and 2.01: with eps = 0.01 both join
    (2.01 <= 2.02) and the colour is their rounded mean; with eps = 0.001 only
    the nearest counts; eps = 0 with equal depths averages the tie."""
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 16, 16, 90.0)
    xyz = np.float32([[2.0, 0.01, 0.01], [2.01, 0.0101, 0.0101], [2.0, 0.012, 0.011]])
    rgb = np.array([[10, 20, 31], [21, 40, 60], [200, 100, 0]], np.uint8)
    key = R.splat(xyz[:2, 0], xyz[:2, 1], xyz[:2, 2], cam.P, 16, 16, 0.1, 1000.0)
    (p,) = np.nonzero(key != EMPTY)
    soft = R.soft_colors(xyz[:2, 0], xyz[:2, 1], xyz[:2, 2], rgb[:2], cam.P, 16, 16, 0.1, 1000.0, key, 0.01)
    # (10 + 21) / 2 = 15.5 -> 16, (20 + 40) / 2 = 30, (31 + 60) / 2 = 45.5 -> 46
    assert soft[p[0]].tolist() == [16, 30, 46, 1]
    soft = R.soft_colors(xyz[:2, 0], xyz[:2, 1], xyz[:2, 2], rgb[:2], cam.P, 16, 16, 0.1, 1000.0, key, 0.001)
    assert soft[p[0]].tolist() == [10, 20, 31, 1]
    key3 = R.splat(xyz[:, 0], xyz[:, 1], xyz[:, 2], cam.P, 16, 16, 0.1, 1000.0)
    soft = R.soft_colors(xyz[:, 0], xyz[:, 1], xyz[:, 2], rgb, cam.P, 16, 16, 0.1, 1000.0, key3, 0.0)
    # points 0 and 2 tie at depth 2.0: (10+200)/2 = 105, (20+100)/2 = 60, (31+0)/2 = 15.5 -> 16
    assert soft[p[0]].tolist() == [105, 60, 16, 1]


def test_soft_zbuffer_brute_force():
    """Per pixel: average of every point landing there within (1 + eps) of the
    nearest depth, searched exhaustively in float64 on a cloud kept off pixel
    borders and with depth gaps far from the threshold."""
    rng = np.random.default_rng(4)
    cam = synth.look_at([0, 0, 0], [10, 0, 0], 12, 10, 60.0)
    xyz = _cloud_off_borders(rng, cam, 600, zrange=(2.0, 3.0))
    rgb = rng.integers(0, 256, xyz.shape, dtype=np.uint8)
    u, v, w = _project64(xyz, cam)
    key = R.splat(xyz[:, 0], xyz[:, 1], xyz[:, 2], cam.P, 12, 10, cam.z_near, cam.z_far)
    eps = 0.05
    soft = R.soft_colors(xyz[:, 0], xyz[:, 1], xyz[:, 2], rgb, cam.P, 12, 10, cam.z_near, cam.z_far, key, eps)
    for py in range(10):
        for px in range(12):
            idx = [j for j in range(len(xyz)) if int(np.floor(u[j])) == px and int(np.floor(v[j])) == py]
            got = soft[py * 12 + px]
            if not idx:
                assert got.tolist() == [0, 0, 0, 0]
                continue
            zmin = min(w[j] for j in idx)
            near = [j for j in idx if w[j] <= zmin * (1 + eps) * (1 - 1e-6)]
            far = [j for j in idx if w[j] > zmin * (1 + eps) * (1 + 1e-6)]
            if len(near) + len(far) != len(idx):
                continue  # a depth within rounding of the threshold
            s = rgb[near].astype(np.int64).sum(0)
            want = (2 * s + len(near)) // (2 * len(near))
            assert got[:3].tolist() == want.tolist() and got[3] == 1


def test_processed_points_counts_points_of_visible_cells():
    """processed_points is the number of points whose own cell is visible:
    checked on a hand-built 3-cell layout and against a per-point loop on a
    random cloud (the cell of each point taken from its coordinates)."""
    from oracle import grid as G
    # cells along x at 1 m: 2 points in cell 0, none in cell 1, 3 in cell 2
    xyz = np.array([[0.1, 0, 0], [0.7, 0, 0], [2.2, 0, 0], [2.5, 0, 0], [2.9, 0, 0]], np.float32)
    g = G.partition(xyz, np.zeros((5, 3), np.uint8), 1.0)
    assert g.dims == (3, 1, 1)
    assert R.processed_points(g, np.array([1, 1, 0], np.uint8)) == 2
    assert R.processed_points(g, np.array([0, 1, 1], np.uint8)) == 3
    assert R.processed_points(g, np.array([1, 0, 1], np.uint8)) == 5
    rng = np.random.default_rng(4)
    pts = rng.uniform(0, 5, (2000, 3)).astype(np.float32)
    g = G.partition(pts, np.zeros((2000, 3), np.uint8), 1.0)
    vis = rng.random(g.n_cells) < 0.4
    want = 0
    for p in pts:
        i = [min(int(np.floor((float(p[a]) - float(g.lo[a])) / 1.0)), g.dims[a] - 1) for a in range(3)]
        want += int(vis[(i[2] * g.dims[1] + i[1]) * g.dims[0] + i[0]])
    assert R.processed_points(g, vis) == want
