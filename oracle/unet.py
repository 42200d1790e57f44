"""Weight-blob parser and float64 U-Net forward pass (oracle; test infrastructure).

Paper: Fig. 1 caption (a fully convolutional U-Net maps the depth-filtered
RGBDA image to the final image) and Method, "U-Net Reconstruction" (the
classic U-Net modified to take RGBDA input; batch normalisation after each
encoder convolution, a training aid).  The paper gives no widths, depths or
normalisation; the readings used here:

  * input x = (r/255, g/255, b/255, A ? D/16 : 0, A) per pixel, with A the
    fill mask and D the z-buffer depth in metres;
  * encoder level l = 0..L-1: two (3x3 conv, zero padding 1, + bias, ReLU);
    after every level but the last, keep the result as skip_l and 2x2 max-pool;
  * decoder level l = L-2..0: nearest x2 upsample, concatenate [skip_l, up],
    two (3x3 conv + bias, ReLU);
  * head: 1x1 conv to 3 channels, no activation;
  * a batch-norm record (conv -> BN -> ReLU) is folded into its convolution:
    W' = W * g / sqrt(var + eps), b' = (b - mean) * g / sqrt(var + eps) + beta.

The 3x3 convolution is written as its definition, a cross-correlation: the
output is the bias plus, for each of the nine taps, the input shifted by that
tap times the tap's C_out x C_in weight matrix (a library matmul as the step).

Pins (tests/test_oracle_unet.py): an independent torch float64 functional
implementation (conv2d / max_pool2d / interpolate / cat), positive
homogeneity f(2x) = 2 f(x) for bias-free nets, an L = 1 net against
scipy.signal.correlate2d, and crop equivalence (an 8-aligned crop with a
margin reproduces the full-image output in its interior).
"""

from __future__ import annotations

import dataclasses
import struct
from typing import List, Tuple

import numpy as np


@dataclasses.dataclass
class Conv:
    W: np.ndarray   # float64 [C_out, C_in, k, k]
    b: np.ndarray   # float64 [C_out]


@dataclasses.dataclass
class UNet:
    widths: Tuple[int, ...]
    in_ch: int
    out_ch: int
    convs: List[Conv]

    @property
    def levels(self) -> int:
        return len(self.widths)


def parse_blob(blob: bytes) -> UNet:
    if blob[:4] != b"LNRU":
        raise ValueError("bad magic")
    version, L, in_ch, out_ch = struct.unpack_from("<4I", blob, 4)
    if version not in (1, 2) or L < 1:
        raise ValueError("bad header")
    off = 20
    widths = struct.unpack_from(f"<{L}I", blob, off)
    off += 4 * L
    convs = []
    for _ in range(4 * L - 1):
        co, ci, k = struct.unpack_from("<3I", blob, off)
        off += 12
        has_bn = 0
        if version == 2:
            (has_bn,) = struct.unpack_from("<I", blob, off)
            off += 4
        nW = co * ci * k * k
        W = np.frombuffer(blob, dtype="<f4", count=nW, offset=off).astype(np.float64).reshape(co, ci, k, k)
        off += 4 * nW
        b = np.frombuffer(blob, dtype="<f4", count=co, offset=off).astype(np.float64)
        off += 4 * co
        if has_bn:
            g, beta, mean, var = (np.frombuffer(blob, dtype="<f4", count=co, offset=off + 4 * co * i)
                                  .astype(np.float64) for i in range(4))
            off += 16 * co
            (eps,) = struct.unpack_from("<f", blob, off)
            off += 4
            scale = g / np.sqrt(var + np.float64(eps))
            W = W * scale[:, None, None, None]
            b = (b - mean) * scale + beta
        convs.append(Conv(W, b))
    if off != len(blob):
        raise ValueError("trailing bytes")
    return UNet(tuple(widths), in_ch, out_ch, convs)


def input_tensor(depth: np.ndarray, rgba: np.ndarray) -> np.ndarray:
    """RGBDA image -> float64 [H, W, 5]."""
    A = (rgba[..., 3] != 0).astype(np.float64)
    x = np.empty(depth.shape + (5,), dtype=np.float64)
    x[..., 0] = rgba[..., 0] / 255.0
    x[..., 1] = rgba[..., 1] / 255.0
    x[..., 2] = rgba[..., 2] / 255.0
    x[..., 3] = np.where(A > 0, depth.astype(np.float64) / 16.0, 0.0)
    x[..., 4] = A
    return x


def conv3x3(x: np.ndarray, c: Conv) -> np.ndarray:
    H, W, _ = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(c.b, (H, W, c.b.shape[0])).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[dy:dy + H, dx:dx + W, :] @ c.W[:, :, dy, dx].T
    return out


def conv1x1(x: np.ndarray, c: Conv) -> np.ndarray:
    return x @ c.W[:, :, 0, 0].T + c.b


def relu(x):
    return np.maximum(x, 0.0)


def maxpool2(x):
    H, W, C = x.shape
    return x.reshape(H // 2, 2, W // 2, 2, C).max(axis=(1, 3))


def up2(x):
    return x.repeat(2, axis=0).repeat(2, axis=1)


def forward_tensor(net: UNet, x: np.ndarray) -> np.ndarray:
    """x float64 [H, W, C_in] -> float64 [C_out, H, W]."""
    L = net.levels
    H, W, _ = x.shape
    if H % (1 << (L - 1)) or W % (1 << (L - 1)):
        raise ValueError("H and W must be divisible by 2^(L-1)")
    it = iter(net.convs)
    skips = []
    for l in range(L):
        x = relu(conv3x3(x, next(it)))
        x = relu(conv3x3(x, next(it)))
        if l < L - 1:
            skips.append(x)
            x = maxpool2(x)
    for l in range(L - 2, -1, -1):
        x = np.concatenate([skips[l], up2(x)], axis=-1)
        x = relu(conv3x3(x, next(it)))
        x = relu(conv3x3(x, next(it)))
    y = conv1x1(x, next(it))
    return np.ascontiguousarray(y.transpose(2, 0, 1))


def forward(net: UNet, depth: np.ndarray, rgba: np.ndarray) -> np.ndarray:
    """RGBDA image -> float64 [3, H, W]."""
    return forward_tensor(net, input_tensor(depth, rgba))


def receptive_margin(levels: int) -> int:
    """A margin (pixels) that covers the receptive radius of the network:
    each 3x3 conv at level l widens it by 2^l full-resolution pixels, and the
    pooling/upsampling grid adds at most 2^L."""
    enc = sum(2 * (1 << l) for l in range(levels))
    dec = sum(2 * (1 << l) for l in range(levels - 1))
    return enc + dec + (1 << levels)


def forward_crop(net: UNet, depth: np.ndarray, rgba: np.ndarray, y0: int, y1: int, x0: int, x1: int):
    """U-Net output over rows [y0, y1) and columns [x0, x1), computed on a crop
    of the input grown by the receptive margin and aligned to 2^(L-1).  The
    interior values equal the full-image ones."""
    L = net.levels
    a = 1 << (L - 1)
    m = receptive_margin(L)
    H, W = depth.shape
    cy0 = max(0, (y0 - m) // a * a)
    cx0 = max(0, (x0 - m) // a * a)
    cy1 = min(H, -(-(y1 + m) // a) * a)
    cx1 = min(W, -(-(x1 + m) // a) * a)
    y = forward(net, depth[cy0:cy1, cx0:cx1], rgba[cy0:cy1, cx0:cx1])
    return y[:, y0 - cy0:y1 - cy0, x0 - cx0:x1 - cx0]


def flops_per_pixel(net: UNet) -> int:
    """Multiply-adds x 2 per full-resolution output pixel."""
    L = net.levels
    it = iter(net.convs)
    macs = 0.0
    for l in range(L):
        for _ in range(2):
            c = next(it)
            macs += c.W.size / 4 ** l
    for l in range(L - 2, -1, -1):
        for _ in range(2):
            c = next(it)
            macs += c.W.size / 4 ** l
    macs += next(it).W.size
    return int(round(2 * macs))
