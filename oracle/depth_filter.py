"""Hierarchical min-pool depth filter (oracle; test infrastructure).

Paper: Method, "Depth filtering", and the Fig. 2 caption.  The image is
min-pooled with a 2x2 kernel and stride 2, n times; then it is upsampled level
by level back to full resolution.  At each upsampling step a Laplacian on the
coarser min-pooled image marks edge pixels; each 2x2 group of children at the
finer level is compared against its parent's depth in the coarser upsampled
image (and, at edge pixels, against the parent's eight neighbours too), with
filter_strength controlling how much survives (smaller = sparser).  Children
that fail stay empty; on every step but the last, empty pixels are filled by
linear interpolation from the coarser upsampled image.

Notation: D_k is the min-pooled image at level k (k = 0 is full resolution,
empty = +inf) and U_k the upsampled image at level k.  The caption counts
upsampling steps i; its "min-pooled(i-1)" / "upsampled(i-1)" are the coarser
level k+1 and "min-pooled(i)" is level k.

Readings where the paper is silent (all arithmetic float32, in this order):
  * odd sizes: H_k = ceil(H_{k-1} / 2); children outside the image are +inf;
  * U_n = D_n;
  * edge test at parent p (level k+1) on D_{k+1}: the 4-neighbour Laplacian
    lap = (((up + down) + left) + right) - 4*D[p] with clamped borders; p is an
    edge if D[p] or any of the four taps is +inf, else iff |lap| > fs * D[p];
  * reference depth: ref = max of U_{k+1} over the in-bounds 3x3 around p at
    edge pixels (a child passes if it passes against the centre or any
    neighbour), else ref = U_{k+1}[p];
  * keep child c iff D_k[c] is finite and D_k[c] <= ref * (1 + fs);
  * U_k[c] = D_k[c] if kept; else, for k > 0, the bilinear value of U_{k+1}
    at c with half-pixel centres and clamped borders:
        y0 = y >> 1, y1 = (y odd) ? min(y0 + 1, Hc - 1) : max(y0 - 1, 0)
        (x0, x1 likewise)
        0.75*(0.75*U[y0,x0] + 0.25*U[y0,x1]) + 0.25*(0.75*U[y1,x0] + 0.25*U[y1,x1]);
    for k = 0 a removed pixel stays empty;
  * output: a pixel that was filled and is kept at level 0 keeps its depth and
    rgba unchanged; every other pixel becomes depth 0, rgba (0, 0, 0, 0).

Parity with the authors' code is unpinned (their implementation details are
in supplementary material that is not available); parity here is with this
reading.  Pins (tests/test_oracle_depth_filter.py): pyramid against the
block-minimum closed form, limiting cases (fs = +inf and n = 0 give the
identity; constant depth survives; all-empty stays empty), invariants
(A_out within A_in, kept pixels unchanged, block-minimum pixels survive),
a two-plane leak scene with a closed-form answer, and two hand-worked 4x4
examples stored under tests/golden/.
"""

from __future__ import annotations

from typing import List

import numpy as np

F32 = np.float32
INF = np.float32(np.inf)


def level_sizes(H: int, W: int, n: int):
    sizes = [(H, W)]
    for _ in range(n):
        h, w = sizes[-1]
        sizes.append(((h + 1) // 2, (w + 1) // 2))
    return sizes


def minpool2(D: np.ndarray) -> np.ndarray:
    """2x2 stride-2 min-pool; a missing row/column (odd size) counts as +inf."""
    h, w = D.shape
    Hc, Wc = (h + 1) // 2, (w + 1) // 2
    pad = np.full((2 * Hc, 2 * Wc), INF, dtype=np.float32)
    pad[:h, :w] = D
    return pad.reshape(Hc, 2, Wc, 2).min(axis=(1, 3))


def pyramid(D0: np.ndarray, n: int) -> List[np.ndarray]:
    levels = [np.asarray(D0, dtype=np.float32)]
    for _ in range(n):
        levels.append(minpool2(levels[-1]))
    return levels


def edge_map(D: np.ndarray, fs) -> np.ndarray:
    """Edge flag per pixel of a min-pooled level (4-neighbour Laplacian, clamped)."""
    h, w = D.shape
    yy = np.arange(h)
    xx = np.arange(w)
    up = D[np.maximum(yy - 1, 0), :]
    down = D[np.minimum(yy + 1, h - 1), :]
    left = D[:, np.maximum(xx - 1, 0)]
    right = D[:, np.minimum(xx + 1, w - 1)]
    any_inf = np.isinf(D) | np.isinf(up) | np.isinf(down) | np.isinf(left) | np.isinf(right)
    with np.errstate(invalid="ignore", over="ignore"):
        lap = (((up + down) + left) + right) - F32(4) * D
        edge = any_inf | (np.abs(lap) > F32(fs) * D)
    return edge


def max3x3(U: np.ndarray) -> np.ndarray:
    """Maximum over the in-bounds 3x3 neighbourhood (out-of-bounds taps ignored)."""
    h, w = U.shape
    pad = np.full((h + 2, w + 2), -INF, dtype=np.float32)
    pad[1:-1, 1:-1] = U
    out = np.full((h, w), -INF, dtype=np.float32)
    for dy in range(3):
        for dx in range(3):
            out = np.maximum(out, pad[dy:dy + h, dx:dx + w])
    return out


def bilerp_up(U: np.ndarray, h: int, w: int) -> np.ndarray:
    """Bilinear value of coarse image U at every pixel of the (h, w) finer level."""
    Hc, Wc = U.shape
    y = np.arange(h)
    x = np.arange(w)
    y0 = y >> 1
    x0 = x >> 1
    y1 = np.where(y & 1, np.minimum(y0 + 1, Hc - 1), np.maximum(y0 - 1, 0))
    x1 = np.where(x & 1, np.minimum(x0 + 1, Wc - 1), np.maximum(x0 - 1, 0))
    U00 = U[y0[:, None], x0[None, :]]
    U01 = U[y0[:, None], x1[None, :]]
    U10 = U[y1[:, None], x0[None, :]]
    U11 = U[y1[:, None], x1[None, :]]
    a, b = F32(0.75), F32(0.25)
    return a * (a * U00 + b * U01) + b * (a * U10 + b * U11)


def upsample_step(Dk: np.ndarray, Dk1: np.ndarray, Uk1: np.ndarray, fs, final: bool):
    """One upsampling step from level k+1 to level k: returns (U_k, keep_k)."""
    h, w = Dk.shape
    edge = edge_map(Dk1, fs)
    ref = np.where(edge, max3x3(Uk1), Uk1)
    thr = ref * (F32(1) + F32(fs))
    y = np.arange(h) >> 1
    x = np.arange(w) >> 1
    thr_c = thr[y[:, None], x[None, :]]
    keep = np.isfinite(Dk) & (Dk <= thr_c)
    if final:
        Uk = np.where(keep, Dk, INF)
    else:
        Uk = np.where(keep, Dk, bilerp_up(Uk1, h, w))
    return Uk.astype(np.float32), keep


def depth_filter(depth: np.ndarray, rgba: np.ndarray, n: int, fs):
    """Filter an RGBDA image.

    depth float32 [H, W] (0 where empty), rgba uint8 [H, W, 4] (alpha 0/1).
    Returns (depth_out, rgba_out, keep0)."""
    depth = np.asarray(depth, dtype=np.float32)
    filled = rgba[..., 3] != 0
    if n == 0:
        return depth.copy(), rgba.copy(), filled.copy()
    D = pyramid(np.where(filled, depth, INF).astype(np.float32), n)
    U = D[n]
    keep = None
    for k in range(n - 1, -1, -1):
        U, keep = upsample_step(D[k], D[k + 1], U, fs, final=(k == 0))
    out_keep = filled & keep
    depth_out = np.where(out_keep, depth, F32(0)).astype(np.float32)
    rgba_out = np.where(out_keep[..., None], rgba, np.uint8(0)).astype(np.uint8)
    return depth_out, rgba_out, out_keep
