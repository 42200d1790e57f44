"""Uniform-grid partition and grid-cell frustum culling (oracle; test infrastructure).

Paper: Method, "Point Cloud Projection" paragraph, and Introduction: the only
preprocessing is a uniform-grid spatial partition that enables view-frustum
culling, so that per-frame work depends on what is visible rather than on
the cloud size.  The paper gives no index formula and no culling test; the
readings used here are:

  * grid origin = componentwise float32 minimum of the cloud; the number of
    cells per axis n_a = max(1, ceil((hi_a - lo_a) / s)) and the cell index
    i_a = min(n_a - 1, floor((x_a - lo_a) / s)), both evaluated in float64;
    cell id c = (i_z * n_y + i_y) * n_x + i_x;
  * points are stably sorted by cell id (the sorted position is the point's
    index everywhere downstream); each cell keeps the tight float32 AABB of
    its points;
  * a cell is culled only when it provably holds no point that passes the
    per-point projection test (see `cull`).  Culling is therefore a pure
    speed-up: a render with culling equals a render without it.

Pins (tests/test_oracle_grid.py): permutation / sortedness / stability
properties that define the unique stable sort, brute-force cell membership,
AABB against per-cell brute force, and cull invariance against an unculled
render over many random cameras (including near-plane and frustum-grazing
ones).
"""

from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Grid:
    lo: np.ndarray          # float32 [3] grid origin
    cell_size: np.float32
    dims: tuple             # (n_x, n_y, n_z)
    perm: np.ndarray        # int64 [N]: sorted position -> input index
    cell_of_sorted: np.ndarray  # int64 [N]
    cell_start: np.ndarray  # int64 [C + 1]
    aabb_lo: np.ndarray     # float32 [C, 3]  (+inf for empty cells)
    aabb_hi: np.ndarray     # float32 [C, 3]  (-inf for empty cells)
    xs: np.ndarray          # float32 [N] sorted SoA coordinates
    ys: np.ndarray
    zs: np.ndarray
    rgb: np.ndarray         # uint8 [N, 3] sorted colours

    @property
    def n_cells(self) -> int:
        return int(self.dims[0] * self.dims[1] * self.dims[2])

    @property
    def counts(self) -> np.ndarray:
        return np.diff(self.cell_start)


def grid_dims(lo: np.ndarray, hi: np.ndarray, cell_size) -> tuple:
    s = np.float64(np.float32(cell_size))
    ext = hi.astype(np.float64) - lo.astype(np.float64)
    return tuple(int(max(1, np.ceil(e / s))) for e in ext)


def cell_ids(xyz: np.ndarray, lo: np.ndarray, dims: tuple, cell_size) -> np.ndarray:
    s = np.float64(np.float32(cell_size))
    rel = xyz.astype(np.float64) - lo.astype(np.float64)[None, :]
    idx = np.floor(rel / s).astype(np.int64)
    idx = np.minimum(idx, np.array(dims, dtype=np.int64)[None, :] - 1)
    return (idx[:, 2] * dims[1] + idx[:, 1]) * dims[0] + idx[:, 0]


def partition(xyz: np.ndarray, rgb: np.ndarray, cell_size: float) -> Grid:
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    lo = xyz.min(axis=0)
    hi = xyz.max(axis=0)
    dims = grid_dims(lo, hi, cell_size)
    C = dims[0] * dims[1] * dims[2]
    cid = cell_ids(xyz, lo, dims, cell_size)
    perm = np.argsort(cid, kind="stable")            # library sort as one step
    cs = cid[perm]
    counts = np.bincount(cs, minlength=C)
    cell_start = np.zeros(C + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_start[1:])
    sx = xyz[perm]
    aabb_lo = np.full((C, 3), np.inf, dtype=np.float32)
    aabb_hi = np.full((C, 3), -np.inf, dtype=np.float32)
    nz = np.nonzero(counts)[0]
    if nz.size:
        starts = cell_start[nz]
        aabb_lo[nz] = np.minimum.reduceat(sx, starts, axis=0)
        aabb_hi[nz] = np.maximum.reduceat(sx, starts, axis=0)
    return Grid(lo, np.float32(cell_size), dims, perm, cs, cell_start, aabb_lo, aabb_hi,
                np.ascontiguousarray(sx[:, 0]), np.ascontiguousarray(sx[:, 1]),
                np.ascontiguousarray(sx[:, 2]), np.ascontiguousarray(rgb[perm]))


# The six half-spaces h(X) >= 0 that a point must satisfy to be splatted,
# written with (a, b, w) = P [X; 1]:
#   w - near, far - w, a, W*w - a, b, H*w - b.
# (a >= 0 and W*w - a > 0 with w > 0 is 0 <= u < W for u = a / w; the same for v.)

SLACK_SCALE = 2.0 ** -20


def halfspaces(P: np.ndarray, W: int, H: int, near, far) -> np.ndarray:
    """float64 [6, 4] coefficients (c_x, c_y, c_z, c_1) of the six half-spaces."""
    p = P.astype(np.float64).reshape(3, 4)
    a, b, w = p[0], p[1], p[2]
    n64, f64 = np.float64(np.float32(near)), np.float64(np.float32(far))
    Wd, Hd = np.float64(W), np.float64(H)
    return np.stack([
        np.array([w[0], w[1], w[2], w[3] - n64]),
        np.array([-w[0], -w[1], -w[2], f64 - w[3]]),
        a,
        np.array([Wd * w[0] - a[0], Wd * w[1] - a[1], Wd * w[2] - a[2], Wd * w[3] - a[3]]),
        b,
        np.array([Hd * w[0] - b[0], Hd * w[1] - b[1], Hd * w[2] - b[2], Hd * w[3] - b[3]]),
    ])


def cull(grid: Grid, P: np.ndarray, W: int, H: int, near, far) -> np.ndarray:
    """Visibility flag per cell (uint8 [C]).

    For every non-empty cell and every half-space, the maximum of h over the
    cell's AABB is exact arithmetic on the corner that maximises each term
    (float64).  The per-point test evaluates a, b, w in float32 with at most
    a few roundings, each below 2^-24 of the sum of the absolute terms; the
    slack 2^-20 * (S_a + S_b + (W + H + 1) * S_w) bounds that error (S_r is
    the sum of |P_r,j * x_j| + |P_r,3| over the AABB's largest magnitudes).
    A cell is culled when some half-space's maximum is below -slack, so no
    point of a culled cell can pass the float32 test."""
    hs = halfspaces(P, W, H, near, far)
    lo = grid.aabb_lo.astype(np.float64)
    hi = grid.aabb_hi.astype(np.float64)
    C = grid.n_cells
    vis = np.zeros(C, dtype=np.uint8)
    nz = grid.counts > 0
    lo, hi = lo[nz], hi[nz]
    p = np.abs(P.astype(np.float64).reshape(3, 4))
    mx = np.maximum(np.abs(lo), np.abs(hi))
    S = [((p[r, 0] * mx[:, 0] + p[r, 1] * mx[:, 1]) + p[r, 2] * mx[:, 2]) + p[r, 3] for r in range(3)]
    slack = SLACK_SCALE * ((S[0] + S[1]) + (np.float64(W) + np.float64(H) + 1.0) * S[2])
    ok = np.ones(lo.shape[0], dtype=bool)
    for c in hs:
        m = ((np.maximum(c[0] * lo[:, 0], c[0] * hi[:, 0])
              + np.maximum(c[1] * lo[:, 1], c[1] * hi[:, 1]))
             + np.maximum(c[2] * lo[:, 2], c[2] * hi[:, 2])) + c[3]
        ok &= ~(m < -slack)
    vis[np.nonzero(nz)[0][ok]] = 1
    return vis
