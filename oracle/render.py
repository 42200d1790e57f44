"""1x1 point projection into a z-buffer, and RGBDA resolve (oracle; test infrastructure).

Paper: Method, "Point Cloud Projection": every point that survives culling is
rasterised as a single pixel to keep all available detail, and a z-buffer
resolves collisions; Fig. 1 caption: the projection yields RGB, depth D and a
binary fill mask A; "U-Net Reconstruction": D is the z-buffer depth and A says
whether a point landed on the pixel.

Readings (the paper leaves these open):
  * hard z-buffer: each pixel keeps its nearest point; ties in depth go to
    the lowest point index, by keeping the minimum of the 64-bit key
    (float32 depth bits << 32) | sorted index (the paper's soft z-buffer,
    which averages colours of points at similar depth, is a separate option);
  * depth = camera-space z, the third row of P;
  * per point, in float32 and in this order:
        a = ((P0*x + P1*y) + P2*z) + P3, b and w likewise from P4..P7, P8..P11;
        accept if near <= w <= far; u = a / w, v = b / w;
        accept if 0 <= u < W and 0 <= v < H; pixel (floor(u), floor(v));
  * resolve: an empty pixel has depth 0 and rgba (0, 0, 0, 0); a filled one
    has the point's depth and rgba (r, g, b, 1).

No culling happens here: the oracle visits every point.  Pins
(tests/test_oracle_render.py): per-pixel exhaustive nearest-point search on
tiny clouds, closed-form single-point positions, duplicate-point tie-breaks,
and an independent float64 projection away from pixel borders.
"""

from __future__ import annotations

import numpy as np

EMPTY_KEY = np.uint64(0xFFFFFFFFFFFFFFFF)


def project(xs, ys, zs, P: np.ndarray, W: int, H: int, near, far):
    """Per point: (valid mask, pixel index, key).  float32 arithmetic, no contraction."""
    P = np.asarray(P, dtype=np.float32)
    xs = np.asarray(xs, dtype=np.float32)
    ys = np.asarray(ys, dtype=np.float32)
    zs = np.asarray(zs, dtype=np.float32)
    a = ((P[0] * xs + P[1] * ys) + P[2] * zs) + P[3]
    b = ((P[4] * xs + P[5] * ys) + P[6] * zs) + P[7]
    w = ((P[8] * xs + P[9] * ys) + P[10] * zs) + P[11]
    valid = (w >= np.float32(near)) & (w <= np.float32(far))
    with np.errstate(divide="ignore", invalid="ignore"):
        u = a / w
        v = b / w
    valid &= (u >= np.float32(0)) & (u < np.float32(W)) & (v >= np.float32(0)) & (v < np.float32(H))
    px = np.where(valid, u, 0).astype(np.int64)
    py = np.where(valid, v, 0).astype(np.int64)
    pix = py * W + px
    j = np.arange(xs.shape[0], dtype=np.uint64)
    key = (w.view(np.uint32).astype(np.uint64) << np.uint64(32)) | j
    return valid, pix, key


def splat(xs, ys, zs, P, W: int, H: int, near, far) -> np.ndarray:
    """z-buffer: key[p] = min over points landing on p of (bits(w) << 32 | j)."""
    valid, pix, key = project(xs, ys, zs, P, W, H, near, far)
    out = np.full(W * H, EMPTY_KEY, dtype=np.uint64)
    np.minimum.at(out, pix[valid], key[valid])
    return out


def resolve(key: np.ndarray, rgb_sorted: np.ndarray):
    """key uint64 [P] -> (depth float32 [P], rgba uint8 [P, 4])."""
    filled = key != EMPTY_KEY
    depth = np.zeros(key.shape[0], dtype=np.float32)
    depth[filled] = (key[filled] >> np.uint64(32)).astype(np.uint32).view(np.float32)
    idx = (key[filled] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    rgba = np.zeros((key.shape[0], 4), dtype=np.uint8)
    rgba[filled, :3] = rgb_sorted[idx]
    rgba[filled, 3] = 1
    return depth, rgba


def soft_colors(xs, ys, zs, rgb_sorted, P, W: int, H: int, near, far, key: np.ndarray, eps) -> np.ndarray:
    """Soft z-buffer colours (Method, "Point Cloud Projection": colours of points
    that arrive at similar depths are averaged, given a small depth threshold).

    Reading: a point joins pixel p's average iff it lands on p and its depth
    w <= zmin * (1 + eps) in float32, zmin being the depth of p's nearest point
    (the hard key); the average of each channel is the integer sum over the
    joined points rounded half up: (2 * sum + count) // (2 * count).
    Returns rgba uint8 [P, 4] (alpha 1 where filled)."""
    valid, pix, k = project(xs, ys, zs, P, W, H, near, far)
    filled = key != EMPTY_KEY
    zmin = np.zeros(key.shape[0], dtype=np.float32)
    zmin[filled] = (key[filled] >> np.uint64(32)).astype(np.uint32).view(np.float32)
    w = (k >> np.uint64(32)).astype(np.uint32).view(np.float32)
    thr = zmin[pix] * (np.float32(1) + np.float32(eps))
    join = valid & (w <= thr)
    sums = np.zeros((key.shape[0], 3), dtype=np.int64)
    count = np.zeros(key.shape[0], dtype=np.int64)
    np.add.at(sums, pix[join], rgb_sorted[join].astype(np.int64))
    np.add.at(count, pix[join], 1)
    rgba = np.zeros((key.shape[0], 4), dtype=np.uint8)
    c = count[filled][:, None]
    rgba[filled, :3] = ((2 * sums[filled] + c) // (2 * c)).astype(np.uint8)
    rgba[filled, 3] = 1
    return rgba


def render(grid, cam):
    """Full projection of a partitioned cloud for one camera: (key, depth, rgba).
    `cam` carries P (float32[12]), width, height, z_near, z_far."""
    key = splat(grid.xs, grid.ys, grid.zs, cam.P, cam.width, cam.height, cam.z_near, cam.z_far)
    depth, rgba = resolve(key, grid.rgb)
    return key, depth, rgba


def processed_points(grid, visible: np.ndarray) -> int:
    """Number of points in visible cells (the points a culled render visits)."""
    return int(grid.counts[visible.astype(bool)].sum())
