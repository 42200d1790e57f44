"""The allocation-free depth filter entry point (lnr_depth_filter_noalloc)
against lnr_depth_filter on the same inputs: bit-identical images on two calls
in a row, the second on a smaller image, with no device memory allocated
through the context; an image whose levels do not fit the fixed scratch is
refused before anything is enqueued."""

import numpy as np
import pytest

from oracle import depth_filter as F
from tests.gpu_util import assert_images_equal, image_from_host, image_to_host

pytestmark = pytest.mark.gpu


def _random_rgbda(H, W, seed):
    rng = np.random.default_rng(seed)
    filled = rng.random((H, W)) < 0.55
    depth = np.where(filled, rng.uniform(0.1, 40, (H, W)), 0).astype(np.float32)
    rgba = rng.integers(0, 256, (H, W, 4)).astype(np.uint8)
    rgba[..., 3] = filled
    rgba[~filled] = 0
    return depth, rgba


def test_noalloc_filter_equals_filter_on_two_calls(lnr, ctx):
    import torch
    fresh = lnr.lnr_context_create(0)
    for (H, W, n, fs, seed) in [(1080, 1920, 5, 0.5, 11), (257, 129, 7, 0.0, 12)]:
        depth, rgba = _random_rgbda(H, W, seed)
        a = image_from_host(lnr, depth, rgba)
        b = image_from_host(lnr, depth, rgba)
        lnr.lnr_depth_filter_noalloc(fresh, a, n, fs)
        lnr.lnr_depth_filter(ctx, b, n, fs)
        torch.cuda.synchronize()
        got, want = image_to_host(a), image_to_host(b)
        assert_images_equal(got, want, f"noalloc vs filter {H}x{W} n={n}")
        wd, wr, _ = F.depth_filter(depth, rgba, n, fs)
        assert_images_equal(got, (None, wd, wr), f"noalloc vs oracle {H}x{W} n={n}")
        assert lnr.lnr_allocated_bytes(fresh) == 0


def test_noalloc_filter_refuses_an_image_beyond_its_scratch(lnr, ctx):
    import torch
    H = W = 4096  # level 1 alone is 4096 x 4096 / 4 floats = 16 MiB, plus level 2
    depth = torch.ones((H, W), dtype=torch.float32, device="cuda")
    rgba = torch.zeros((H, W, 4), dtype=torch.uint8, device="cuda")
    rgba[..., 3] = 1
    img = lnr.Image.from_tensors(depth, rgba, None)
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_depth_filter_noalloc(ctx, img, 2, 0.5)
    assert e.value.status == lnr.LNR_E_INVALID_ARG
    assert "allocation-free" in str(e.value)
    torch.cuda.synchronize()
    assert bool((depth == 1).all()) and bool((rgba[..., 3] == 1).all())
