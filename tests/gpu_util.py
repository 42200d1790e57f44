"""Helpers shared by the GPU tests (host-side marshalling and comparisons)."""

import numpy as np
import pytest

# lnr_precision values (include/lnr.h) and the U-Net's max-abs bound against
# the float64 oracle in each: float32 1e-4, the 16-bit formats 2e-2, the e4m3
# formats 8e-2
FP32, BF16, FP8_E4M3, BF16X3, FP16, FP8_E4M3X3 = 0, 1, 2, 3, 4, 5
BOUND = {FP32: 1e-4, BF16: 2e-2, FP8_E4M3: 8e-2, BF16X3: 2e-2, FP16: 2e-2, FP8_E4M3X3: 8e-2}
NAMES = {FP32: "fp32", BF16: "bf16", FP8_E4M3: "fp8-e4m3", BF16X3: "bf16x3", FP16: "fp16",
         FP8_E4M3X3: "fp8-e4m3x3"}
# precisions whose rounding is known to exceed the bound on these He-initialised
# networks, by a float emulation before any kernel: plain bf16 (a 7-bit
# fraction on every weight and activation: about 3e-2 max-abs on the room
# frames and 3.4e-2 on a full 1080p frame) and plain e4m3 (a 3-bit fraction:
# about 0.48 on a room frame, and 0.14-0.24 with e4m3 in any single layer
# alone); held to their bounds all the same and reported as expected failures
OUT_OF_BOUND = {BF16, FP8_E4M3}
# every U-Net precision the library builds, in test order
UNET_PRECISIONS = [FP32, BF16X3, FP16, FP8_E4M3X3, BF16, FP8_E4M3]


def check_unet_error(prec, err, what=""):
    """Assert the U-Net max-abs error is within its precision's bound."""
    if err <= BOUND[prec]:
        return
    msg = f"{NAMES[prec]} {what}: max-abs {err:.3e} exceeds the bound {BOUND[prec]:.0e}"
    if prec in OUT_OF_BOUND:
        pytest.xfail(msg)
    raise AssertionError(msg)


def image_to_host(img):
    key = None if img.key is None else img.key.cpu().numpy().view(np.uint64).copy()
    return key, img.depth.cpu().numpy().copy(), img.rgba.cpu().numpy().copy()


def image_from_host(lnr, depth, rgba, key=None):
    import torch
    d = torch.from_numpy(np.ascontiguousarray(depth, dtype=np.float32)).cuda()
    r = torch.from_numpy(np.ascontiguousarray(rgba, dtype=np.uint8)).cuda()
    k = None if key is None else torch.from_numpy(np.ascontiguousarray(key).view(np.int64)).cuda()
    return lnr.Image.from_tensors(d, r, k)


def render_gpu(lnr, ctx, cloud, cam, flags=0):
    import torch
    img = lnr.Image(cam.height, cam.width)
    lnr.lnr_render(ctx, cloud, cam, img, flags)
    torch.cuda.synchronize()
    return img


def assert_images_equal(got, want, what=""):
    gk, gd, gr = got
    wk, wd, wr = want
    if wk is not None and gk is not None:
        bad = np.nonzero(gk.reshape(-1) != wk.reshape(-1))[0]
        assert bad.size == 0, f"{what}: {bad.size} key mismatches, first at {bad[:5]}"
    assert np.array_equal(gd.reshape(-1).view(np.uint32), wd.reshape(-1).view(np.uint32)), f"{what}: depth differs"
    assert np.array_equal(gr.reshape(-1), wr.reshape(-1)), f"{what}: rgba differs"
