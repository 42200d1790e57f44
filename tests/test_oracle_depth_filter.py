"""Pins of the oracle's min-pool pyramid and depth filter (CPU only)."""

import json
import os

import numpy as np
import pytest

from oracle import depth_filter as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "depth_filter_examples.json")
INF = np.float32(np.inf)


def _random_rgbda(rng, H, W, fill=0.6, lo=0.5, hi=30.0):
    filled = rng.random((H, W)) < fill
    depth = np.where(filled, rng.uniform(lo, hi, (H, W)), 0).astype(np.float32)
    rgba = np.zeros((H, W, 4), np.uint8)
    rgba[..., :3] = rng.integers(0, 256, (H, W, 3))
    rgba[..., 3] = filled
    rgba[~filled] = 0
    return depth, rgba


@pytest.mark.parametrize("H,W,n", [(1, 1, 0), (5, 7, 3), (16, 16, 4), (27, 40, 5), (33, 1, 5)])
def test_pyramid_is_the_block_minimum(H, W, n):
    rng = np.random.default_rng(H * 100 + W)
    D0 = np.where(rng.random((H, W)) < 0.5, rng.uniform(0.1, 9, (H, W)), np.inf).astype(np.float32)
    levels = F.pyramid(D0, n)
    for k, Dk in enumerate(levels):
        b = 1 << k
        assert Dk.shape == (-(-H // b), -(-W // b))
        for y in range(Dk.shape[0]):
            for x in range(Dk.shape[1]):
                blk = D0[y * b:(y + 1) * b, x * b:(x + 1) * b]
                assert Dk[y, x] == blk.min()
        # every child >= its parent, and the global minimum is the same on every level
        if k:
            prev = levels[k - 1]
            par = Dk[np.arange(prev.shape[0])[:, None] >> 1, np.arange(prev.shape[1])[None, :] >> 1]
            assert np.all(prev >= par)
        assert Dk.min() == D0.min()


def test_golden_examples():
    with open(GOLDEN) as f:
        data = json.load(f)
    for ex in data["examples"]:
        d = np.array([[np.nan if v is None else v for v in row] for row in ex["depth"]], dtype=np.float64)
        filled = ~np.isnan(d)
        depth = np.where(filled, d, 0).astype(np.float32)
        rgba = np.zeros(depth.shape + (4,), np.uint8)
        rgba[..., 0] = 7
        rgba[..., 3] = filled
        rgba[~filled] = 0
        dout, rout, keep = F.depth_filter(depth, rgba, ex["n"], ex["fs"])
        assert keep.astype(int).tolist() == ex["mask"], ex["name"]
        assert np.array_equal(dout[keep], depth[keep])
        assert np.all(dout[~keep] == 0) and np.all(rout[~keep] == 0)


@pytest.mark.parametrize("seed,H,W,n", [(0, 32, 32, 3), (1, 45, 61, 4), (2, 64, 48, 5)])
def test_limits_and_invariants(seed, H, W, n):
    rng = np.random.default_rng(seed)
    depth, rgba = _random_rgbda(rng, H, W)
    # filter_strength = +inf keeps everything; n = 0 is the identity
    for args in ((n, np.inf), (0, 0.5), (0, 0.0)):
        d2, r2, _ = F.depth_filter(depth, rgba, *args)
        assert np.array_equal(d2, depth) and np.array_equal(r2, rgba)
    filled = rgba[..., 3] != 0
    D0 = np.where(filled, depth, INF)
    B = 1 << n
    blockmin = F.pyramid(D0, n)[n]
    bm_full = blockmin[np.arange(H)[:, None] // B, np.arange(W)[None, :] // B]
    for fs in (0.0, 0.1, 0.5, 2.0):
        d2, r2, keep = F.depth_filter(depth, rgba, n, fs)
        a_out = r2[..., 3] != 0
        assert np.all(~a_out | filled)                     # A_out within A_in
        assert np.array_equal(d2[a_out], depth[a_out])     # kept pixels unchanged
        assert np.array_equal(r2[a_out], rgba[a_out])
        assert np.all(d2[~a_out] == 0) and np.all(r2[~a_out] == 0)
        assert np.all(a_out[filled & (D0 == bm_full)])     # block minima always survive


@pytest.mark.parametrize("fs", [0.0, 0.5, 3.0])
def test_constant_depth_and_empty(fs):
    H, W = 40, 24
    rgba = np.full((H, W, 4), 9, np.uint8)
    rgba[..., 3] = 1
    depth = np.full((H, W), 3.25, np.float32)
    d2, r2, _ = F.depth_filter(depth, rgba, 3, fs)
    assert np.array_equal(d2, depth) and np.array_equal(r2, rgba)
    z = np.zeros((H, W), np.float32)
    e = np.zeros((H, W, 4), np.uint8)
    d2, r2, keep = F.depth_filter(z, e, 3, fs)
    assert not keep.any() and not r2.any() and not d2.any()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_two_plane_leak_scene(n):
    """Foreground at depth 2 with checkerboard holes in front of a background at 8:
    inside the foreground (away from its border) all leaked background pixels
    are removed and every foreground pixel kept; far from the foreground every
    background pixel is kept.  Power-of-two depths keep interpolation exact."""
    H, W = 160, 192
    depth = np.full((H, W), 8.0, np.float32)
    y0, y1, x0, x1 = 32, 128, 48, 176
    yy, xx = np.mgrid[0:H, 0:W]
    fg = (yy >= y0) & (yy < y1) & (xx >= x0) & (xx < x1) & ((yy + xx) % 2 == 0)
    depth[fg] = 2.0
    rgba = np.ones((H, W, 4), np.uint8)
    _, _, keep = F.depth_filter(depth, rgba, n, 0.5)
    m = (1 << (n + 1)) + 4
    interior = (yy >= y0 + m) & (yy < y1 - m) & (xx >= x0 + m) & (xx < x1 - m)
    assert np.all(keep[interior & fg])
    assert not np.any(keep[interior & ~fg])
    far = (yy < y0 - m) | (xx < x0 - m)
    assert np.all(keep[far])


def test_sizes_ladder():
    assert F.level_sizes(1080, 1920, 5) == [(1080, 1920), (540, 960), (270, 480), (135, 240), (68, 120), (34, 60)]


def test_edge_map_hand_values():
    """3x3 ramp 1..9, fs = 0.25, clamped borders.  |lap| by hand:
    [[4, 3, 2], [1, 0, 1], [2, 3, 4]] against fs*D = [[.25, .5, .75], [1, 1.25, 1.5],
    [1.75, 2, 2.25]]; (1, 0) has |lap| == fs*D exactly and is not an edge."""
    D = np.arange(1, 10, dtype=np.float32).reshape(3, 3)
    assert F.edge_map(D, 0.25).astype(int).tolist() == [[1, 1, 1], [0, 0, 0], [1, 1, 1]]
    D2 = D.copy()
    D2[0, 2] = np.inf  # an empty tap makes the pixel and its 4-neighbours edges
    e = F.edge_map(D2, 100.0).astype(int).tolist()
    assert e == [[0, 1, 1], [0, 0, 1], [0, 0, 0]]


def test_bilinear_fill_matches_torch_bilinear():
    """With half-pixel centres and clamped borders the fill is the standard x2
    bilinear upsample (align_corners=False); dyadic inputs keep both exact."""
    import torch
    import torch.nn.functional as Fn
    rng = np.random.default_rng(0)
    for (hc, wc) in [(2, 2), (3, 5), (7, 4)]:
        U = (rng.integers(1, 64, (hc, wc)) / 4.0).astype(np.float32)
        ref = Fn.interpolate(torch.tensor(U)[None, None], scale_factor=2, mode="bilinear",
                             align_corners=False)[0, 0].numpy()
        for (h, w) in [(2 * hc, 2 * wc), (2 * hc - 1, 2 * wc - 1)]:
            assert np.array_equal(F.bilerp_up(U, h, w), ref[:h, :w])
    U = np.array([[1, 2], [3, 4]], np.float32)
    assert F.bilerp_up(U, 4, 4)[1].tolist() == [1.5, 1.75, 2.25, 2.5]


def test_max3x3_hand_values():
    U = np.array([[1, 5, 2], [0, 0, 0], [3, 0, 9]], np.float32)
    assert F.max3x3(U).tolist() == [[5, 5, 5], [5, 9, 9], [3, 9, 9]]
