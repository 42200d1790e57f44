"""Pins of the oracle's grid partition and frustum culling (CPU only)."""

import numpy as np
import pytest

import synth
from oracle import grid as G
from oracle import render as R


def _random_cloud(rng, n, spread=5.0):
    xyz = (rng.standard_normal((n, 3)) * spread).astype(np.float32)
    rgb = rng.integers(0, 256, (n, 3), dtype=np.uint8)
    return xyz, rgb


@pytest.mark.parametrize("seed,n,s", [(0, 1, 0.5), (1, 17, 1.0), (2, 5000, 0.7), (3, 20000, 2.5)])
def test_partition_is_the_stable_sort_by_cell(seed, n, s):
    rng = np.random.default_rng(seed)
    xyz, rgb = _random_cloud(rng, n)
    # duplicate some points so equal keys and equal coordinates occur
    if n > 10:
        xyz[n // 2:n // 2 + 5] = xyz[:5]
    g = G.partition(xyz, rgb, s)
    perm = g.perm
    # a permutation
    assert np.array_equal(np.sort(perm), np.arange(n))
    # cell of each sorted point, recomputed by brute force from the box test
    s64 = np.float64(np.float32(s))
    lo = xyz.min(0).astype(np.float64)
    dims = np.array(g.dims)
    for j in range(0, n, max(1, n // 500)):
        p = xyz[perm[j]].astype(np.float64)
        c = g.cell_of_sorted[j]
        ix, iy, iz = c % dims[0], (c // dims[0]) % dims[1], c // (dims[0] * dims[1])
        for a, i in enumerate((ix, iy, iz)):
            cl = lo[a] + i * s64
            assert cl - 1e-9 <= p[a]
            assert p[a] < cl + s64 + 1e-9 or i == dims[a] - 1
    # non-decreasing cells, increasing original index inside a cell => unique stable order
    cs = g.cell_of_sorted
    assert np.all(np.diff(cs) >= 0)
    same = np.diff(cs) == 0
    assert np.all(np.diff(perm)[same] > 0)
    # CSR offsets
    assert g.cell_start[0] == 0 and g.cell_start[-1] == n
    assert np.array_equal(np.diff(g.cell_start), np.bincount(cs, minlength=g.n_cells))
    # sorted SoA and colours follow perm
    assert np.array_equal(g.xs, xyz[perm, 0]) and np.array_equal(g.zs, xyz[perm, 2])
    assert np.array_equal(g.rgb, rgb[perm])


def test_grid_dims_and_extremes():
    xyz = np.array([[0, 0, 0], [1.0, 2.0, 0.0], [1.0, 2.0, 0.0]], dtype=np.float32)
    g = G.partition(xyz, np.zeros((3, 3), np.uint8), 0.5)
    assert g.dims == (2, 4, 1)  # ceil(1/0.5), ceil(2/0.5), max(1, 0)
    # the max point lies on the far face and is clamped into the last cell
    assert g.cell_of_sorted[-1] == (0 * 4 + 3) * 2 + 1


def test_aabb_is_tight(room_scene):
    g = G.partition(room_scene.xyz, room_scene.rgb, 0.5)
    cnt = g.counts
    for c in np.nonzero(cnt)[0][::37]:
        a, b = g.cell_start[c], g.cell_start[c + 1]
        pts = np.stack([g.xs[a:b], g.ys[a:b], g.zs[a:b]], 1)
        assert np.array_equal(g.aabb_lo[c], pts.min(0))
        assert np.array_equal(g.aabb_hi[c], pts.max(0))
    empty = cnt == 0
    assert np.all(np.isinf(g.aabb_lo[empty]))


def _grazing_cameras(rng, xyz, n):
    """Cameras whose image border or near plane passes through cloud points."""
    cams = []
    W, H = 64, 48
    for _ in range(n):
        eye = xyz[rng.integers(len(xyz))].astype(np.float64) + rng.normal(0, 0.3, 3)
        tgt = xyz[rng.integers(len(xyz))].astype(np.float64)
        if np.linalg.norm(tgt - eye) < 0.2:
            continue
        fov = rng.uniform(20, 120)
        near = float(rng.choice([0.1, 0.5, 2.0]))
        far = float(rng.choice([1000.0, 3.0, 6.0]))
        cam = synth.look_at(eye, tgt, W, H, fov, near, far)
        cams.append(cam)
    return cams


def test_cull_is_conservative_many_cameras(room_scene):
    """No point of a culled cell passes the per-point projection test, over many
    random cameras (eye near the cloud, near planes that cut through it, small far
    planes, narrow and wide fields of view).  Hence a culled render equals the
    unculled one."""
    rng = np.random.default_rng(5)
    sub = room_scene.xyz[::10]
    g = G.partition(sub, room_scene.rgb[::10], 0.5)
    cams = _grazing_cameras(rng, sub, 1200)
    culled_total = 0
    for cam in cams:
        vis = G.cull(g, cam.P, cam.width, cam.height, cam.z_near, cam.z_far)
        valid, _, _ = R.project(g.xs, g.ys, g.zs, cam.P, cam.width, cam.height, cam.z_near, cam.z_far)
        point_vis = np.repeat(vis, g.counts).astype(bool)
        assert not np.any(valid & ~point_vis)
        culled_total += int((g.counts > 0).sum() - vis.sum())
    assert culled_total > 0  # culling does remove cells


def test_cull_exact_border_points():
    """Points placed exactly on the image border and the near/far planes: the
    cells that hold accepted points are never culled."""
    cam = synth.look_at([0, 0, 0], [1, 0, 0], 32, 32, 90.0, 0.5, 4.0)
    P = cam.P.astype(np.float64).reshape(3, 4)
    pts = []
    for depth in (0.5, 1.0, 4.0):
        for u in (0.0, 31.999, 16.0):
            for v in (0.0, 31.999, 16.0):
                # invert the projection in float64 for this depth
                A = np.array([P[0, :3] - u * P[2, :3], P[1, :3] - v * P[2, :3], P[2, :3]])
                rhs = np.array([u * P[2, 3] - P[0, 3], v * P[2, 3] - P[1, 3], depth - P[2, 3]])
                pts.append(np.linalg.solve(A, rhs))
    xyz = np.array(pts, dtype=np.float32)
    g = G.partition(xyz, np.zeros_like(xyz, dtype=np.uint8), 0.25)
    vis = G.cull(g, cam.P, 32, 32, 0.5, 4.0)
    valid, _, _ = R.project(g.xs, g.ys, g.zs, cam.P, 32, 32, 0.5, 4.0)
    assert valid.sum() > 0
    assert np.all(np.repeat(vis, g.counts).astype(bool)[valid])


def test_cull_far_behind_camera_is_culled(room_scene):
    g = G.partition(room_scene.xyz, room_scene.rgb, 0.5)
    # camera outside the room looking away from it
    cam = synth.look_at([-5, 4, 1.5], [-10, 4, 1.5], 64, 64, 70.0)
    vis = G.cull(g, cam.P, 64, 64, cam.z_near, cam.z_far)
    assert vis.sum() == 0
