"""Helpers shared by the GPU tests (host-side marshalling and comparisons)."""

import numpy as np


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
