"""Pins of the oracle's float64 U-Net (CPU only).

The independent reference here is PyTorch's float64 functional ops on the CPU
(conv2d, max_pool2d, interpolate, cat), which share no code with the oracle's
tap-by-tap numpy formulation."""

import struct

import numpy as np
import pytest
import torch
import torch.nn.functional as Fn
from scipy.signal import correlate2d

import synth
from oracle import unet as U


def _torch_unet(blob, x_hwc, fold_bn=True):
    """Independent float64 forward pass from the raw blob (NCHW, torch ops)."""
    version, L, in_ch, out_ch = struct.unpack_from("<4I", blob, 4)
    off = 20 + 4 * L
    layers = []
    for _ in range(4 * L - 1):
        co, ci, k = struct.unpack_from("<3I", blob, off)
        off += 12
        has_bn = 0
        if version == 2:
            has_bn = struct.unpack_from("<I", blob, off)[0]
            off += 4
        W = torch.tensor(np.frombuffer(blob, "<f4", co * ci * k * k, off).reshape(co, ci, k, k), dtype=torch.float64)
        off += 4 * co * ci * k * k
        b = torch.tensor(np.frombuffer(blob, "<f4", co, off), dtype=torch.float64)
        off += 4 * co
        bn = None
        if has_bn:
            arr = [torch.tensor(np.frombuffer(blob, "<f4", co, off + 4 * co * i), dtype=torch.float64) for i in range(4)]
            off += 16 * co
            eps = struct.unpack_from("<f", blob, off)[0]
            off += 4
            bn = (arr, eps)
        layers.append((W, b, bn))
    it = iter(layers)

    def conv(x):
        W, b, bn = next(it)
        y = Fn.conv2d(x, W, b, padding=W.shape[-1] // 2)
        if bn is not None:
            (g, beta, mean, var), eps = bn
            y = Fn.batch_norm(y, mean, var, g, beta, training=False, eps=eps)
        return y

    x = torch.tensor(x_hwc, dtype=torch.float64).permute(2, 0, 1)[None]
    skips = []
    for l in range(L):
        x = torch.relu(conv(x))
        x = torch.relu(conv(x))
        if l < L - 1:
            skips.append(x)
            x = Fn.max_pool2d(x, 2)
    for l in range(L - 2, -1, -1):
        x = torch.cat([skips[l], Fn.interpolate(x, scale_factor=2, mode="nearest")], 1)
        x = torch.relu(conv(x))
        x = torch.relu(conv(x))
    return conv(x)[0].numpy()


@pytest.mark.parametrize("widths,H,W,bias,bn", [
    ((4,), 6, 10, "uniform", False),
    ((8, 16), 16, 12, "uniform", False),
    ((16, 32, 64), 32, 24, "zero", False),
    ((8, 8, 16, 16), 24, 40, "uniform", True),
])
def test_matches_torch_float64(widths, H, W, bias, bn):
    rng = np.random.default_rng(len(widths))
    blob = synth.make_unet_blob(widths, seed=3, bias=bias, batchnorm=bn)
    net = U.parse_blob(blob)
    x = rng.uniform(0, 1, (H, W, 5))
    y = U.forward_tensor(net, x)
    ref = _torch_unet(blob, x)
    assert y.shape == (3, H, W)
    assert np.max(np.abs(y - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_positive_homogeneity():
    blob = synth.make_unet_blob((8, 16, 32), seed=1, bias="zero")
    net = U.parse_blob(blob)
    x = np.random.default_rng(0).uniform(0, 1, (16, 16, 5))
    assert np.array_equal(U.forward_tensor(net, 2.0 * x), 2.0 * U.forward_tensor(net, x))


def test_single_level_is_two_correlations_and_a_pointwise_map():
    blob = synth.make_unet_blob((3,), seed=5, bias="uniform")
    net = U.parse_blob(blob)
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, (9, 11, 5))

    def conv(x, c):
        out = np.zeros((c.W.shape[0],) + x.shape[:2])
        for o in range(c.W.shape[0]):
            for i in range(c.W.shape[1]):
                out[o] += correlate2d(x[..., i], c.W[o, i], mode="same", boundary="fill")
            out[o] += c.b[o]
        return out.transpose(1, 2, 0)

    h = np.maximum(conv(x, net.convs[0]), 0)
    h = np.maximum(conv(h, net.convs[1]), 0)
    head = net.convs[2]
    y = np.einsum("hwc,oc->ohw", h, head.W[:, :, 0, 0]) + head.b[:, None, None]
    assert np.max(np.abs(U.forward_tensor(net, x) - y)) < 1e-12


def test_input_tensor_definition():
    depth = np.array([[3.2, 5.0]], np.float32)  # depth of an empty pixel is ignored
    rgba = np.array([[[255, 51, 0, 1], [0, 0, 0, 0]]], np.uint8)
    x = U.input_tensor(depth, rgba)
    assert np.allclose(x[0, 0], [1.0, 0.2, 0.0, np.float64(np.float32(3.2)) / 16, 1.0], rtol=0, atol=1e-15)
    assert np.all(x[0, 1] == 0)


@pytest.mark.parametrize("widths,H,W", [
    ((4, 8, 8), 96, 128),
    # the depths the full-size (4 levels) and 4K (5 levels) GPU tests compare on crops
    ((4, 6, 8, 8), 176, 208),
    ((4, 4, 6, 6, 8), 352, 384),
])
def test_crop_reproduces_full_image_interior(widths, H, W):
    """forward_crop (a crop grown by receptive_margin and aligned to 2^(L-1))
    equals the full-image forward pass on windows at the corners, the edges
    and the interior; with half the margin the interior window differs, so the
    comparison would catch a margin that is too small."""
    L = len(widths)
    blob = synth.make_unet_blob(widths, seed=2, bias="uniform")
    net = U.parse_blob(blob)
    rng = np.random.default_rng(3 + L)
    depth = rng.uniform(0.5, 10, (H, W)).astype(np.float32)
    rgba = rng.integers(0, 256, (H, W, 4)).astype(np.uint8)
    rgba[..., 3] = rng.random((H, W)) < 0.7
    full = U.forward(net, depth, rgba)
    m = U.receptive_margin(L)
    assert min(H, W) > 2 * m + 16  # the interior window has a real crop around it
    windows = [(0, 8, 0, 16), (H - 6, H, W - 8, W), (0, 16, W - 16, W), (H - 16, H, 0, 16),
               (H // 2 - 3, H // 2 + 5, W // 2 - 7, W // 2 + 9)]
    for (y0, y1, x0, x1) in windows:
        part = U.forward_crop(net, depth, rgba, y0, y1, x0, x1)
        assert np.max(np.abs(part - full[:, y0:y1, x0:x1])) < 1e-12, (L, y0, x0)
    if L >= 4:
        y0, y1, x0, x1 = windows[-1]
        orig = U.receptive_margin
        try:
            U.receptive_margin = lambda levels: orig(levels) // 2
            part = U.forward_crop(net, depth, rgba, y0, y1, x0, x1)
        finally:
            U.receptive_margin = orig
        assert np.max(np.abs(part - full[:, y0:y1, x0:x1])) > 1e-9


def test_parser_rejects_bad_blobs():
    blob = synth.make_unet_blob((4,), seed=0)
    with pytest.raises(ValueError):
        U.parse_blob(b"XXXX" + blob[4:])
    with pytest.raises(ValueError):
        U.parse_blob(blob + b"\0")


def test_flop_count_matches_the_convolutions_a_forward_pass_runs(monkeypatch):
    """flops_per_pixel x H x W equals 2 x the multiply-adds of the convolutions
    that a forward pass actually calls, counted from their operand shapes."""
    widths = (4, 8, 12, 16)
    net = U.parse_blob(synth.make_unet_blob(widths, seed=0))
    H, W = 48, 64
    macs = []
    c3, c1 = U.conv3x3, U.conv1x1

    def count3(x, c):
        macs.append(x.shape[0] * x.shape[1] * c.W.shape[0] * c.W.shape[1] * 9)
        return c3(x, c)

    def count1(x, c):
        macs.append(x.shape[0] * x.shape[1] * c.W.shape[0] * c.W.shape[1])
        return c1(x, c)

    monkeypatch.setattr(U, "conv3x3", count3)
    monkeypatch.setattr(U, "conv1x1", count1)
    depth = np.ones((H, W), np.float32)
    rgba = np.ones((H, W, 4), np.uint8)
    U.forward(net, depth, rgba)
    assert len(macs) == 4 * len(widths) - 1
    assert U.flops_per_pixel(net) * H * W == 2 * sum(macs)
