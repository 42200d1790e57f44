"""GPU parity of the depth filter against the oracle (bit-exact)."""

import json
import os

import numpy as np
import pytest

from oracle import depth_filter as F
from oracle import render as R
from tests.gpu_util import assert_images_equal, image_from_host, image_to_host, render_gpu

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "depth_filter_examples.json")


def _filter_gpu(lnr, ctx, depth, rgba, n, fs):
    import torch
    img = image_from_host(lnr, depth, rgba)
    lnr.lnr_depth_filter(ctx, img, n, fs)
    torch.cuda.synchronize()
    return image_to_host(img)


def test_golden_examples(lnr, ctx):
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
        _, gd, gr = _filter_gpu(lnr, ctx, depth, rgba, ex["n"], ex["fs"])
        assert (gr[..., 3] != 0).astype(int).tolist() == ex["mask"], ex["name"]


@pytest.mark.parametrize("H,W,n", [(1, 1, 0), (2, 2, 1), (7, 5, 2), (64, 64, 6), (135, 240, 5), (257, 129, 7),
                                   (1080, 1920, 5), (33, 1000, 5)])
@pytest.mark.parametrize("fs", [0.0, 0.5, 2.0, np.inf])
def test_random_images(lnr, ctx, H, W, n, fs):
    rng = np.random.default_rng(H * 7 + W + n)
    filled = rng.random((H, W)) < 0.55
    depth = np.where(filled, rng.uniform(0.1, 40, (H, W)), 0).astype(np.float32)
    rgba = rng.integers(0, 256, (H, W, 4)).astype(np.uint8)
    rgba[..., 3] = filled
    rgba[~filled] = 0
    want_d, want_r, _ = F.depth_filter(depth, rgba, n, fs)
    got = _filter_gpu(lnr, ctx, depth, rgba, n, fs)
    assert_images_equal(got, (None, want_d, want_r), f"{H}x{W} n={n} fs={fs}")


def test_rendered_frames(lnr, ctx, room_cloud, room_grid, room_cams):
    import torch
    for i, cam in enumerate(room_cams):
        img = render_gpu(lnr, ctx, room_cloud, cam)
        lnr.lnr_depth_filter(ctx, img, 4, 0.5)
        torch.cuda.synchronize()
        key, depth, rgba = R.render(room_grid, cam)
        H, W = cam.height, cam.width
        wd, wr, _ = F.depth_filter(depth.reshape(H, W), rgba.reshape(H, W, 4), 4, 0.5)
        gk, gd, gr = image_to_host(img)
        assert np.array_equal(gk, key), "the filter must not touch the key buffer"
        assert_images_equal((None, gd, gr), (None, wd, wr), f"frame {i}")


def test_rejects_bad_levels(lnr, ctx):
    depth = np.zeros((8, 8), np.float32)
    rgba = np.zeros((8, 8, 4), np.uint8)
    img = image_from_host(lnr, depth, rgba)
    for n, fs in [(4, 0.5), (-1, 0.5), (2, -0.1), (2, float("nan"))]:
        with pytest.raises(lnr.LnrError) as e:
            lnr.lnr_depth_filter(ctx, img, n, fs)
        assert e.value.status == lnr.LNR_E_INVALID_ARG
