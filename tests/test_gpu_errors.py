"""Error paths under injected device-allocation failures (lnr_debug_fail_allocation).

For every entry point that allocates: each of its allocations in turn is made
to fail; the call must return LNR_E_OUT_OF_MEMORY, free what it took (the
library's allocation count returns to where it was, or, for a context's
grow-only scratch, to what a clean run leaves), and leave caller buffers
untouched.  The failures are injected on the host, so no kernel misbehaves."""

import numpy as np
import pytest

import synth
from tests.gpu_util import FP16, FP32, BF16X3, FP8_E4M3X3

pytestmark = pytest.mark.gpu


def _sweep(lnr, ctx, call, limit=64):
    """Run call() with the n-th allocation failing, n = 0, 1, ... until it
    succeeds; return the number of failing runs."""
    for n in range(limit):
        lnr.lnr_debug_fail_allocation(ctx, n)
        try:
            call()
        except lnr.LnrError as e:
            assert e.status == lnr.LNR_E_OUT_OF_MEMORY, str(e)
            assert "injected" in lnr.lnr_last_error(ctx)
            yield n
            continue
        finally:
            lnr.lnr_debug_fail_allocation(ctx, -1)
        return
    raise AssertionError("the call never succeeded")


def test_cloud_and_network_loads_free_everything_on_failure(lnr, room_scene):
    ctx = lnr.lnr_context_create(0)
    base = lnr.lnr_allocated_bytes(ctx)
    xyz, rgb = room_scene.xyz[:50000], room_scene.rgb[:50000]
    fails = 0
    for _ in _sweep(lnr, ctx, lambda: lnr.lnr_cloud_load(ctx, xyz, rgb, 0.5)):
        assert lnr.lnr_allocated_bytes(ctx) == base
        fails += 1
    assert fails >= 5
    blob = synth.make_unet_blob((16, 32), seed=0)
    for prec in (FP32, BF16X3, FP16, FP8_E4M3X3):
        fails = 0
        for _ in _sweep(lnr, ctx, lambda: lnr.lnr_unet_load(ctx, blob, prec)):
            assert lnr.lnr_allocated_bytes(ctx) == base
            fails += 1
        assert fails >= 4


def _sentinel_image(lnr, H, W):
    import torch
    img = lnr.Image(H, W)
    img.key.fill_(0x5A5A5A5A5A5A5A5A)
    img.depth.fill_(-3.25)
    img.rgba.fill_(0xA5)
    torch.cuda.synchronize()
    return img


def _untouched(img):
    import torch
    torch.cuda.synchronize()
    return (bool((img.key == 0x5A5A5A5A5A5A5A5A).all()) and bool((img.depth == -3.25).all())
            and bool((img.rgba == 0xA5).all()))


@pytest.mark.parametrize("soft", [False, True])
def test_render_filter_reconstruct_leave_outputs_untouched(lnr, room_cloud, room_cams, soft):
    import torch
    cam = room_cams[3]
    H, W = cam.height, cam.width
    blob = synth.make_unet_blob((16, 32, 64), seed=0)
    # scratch a clean run leaves in a fresh context
    clean = lnr.lnr_context_create(0)
    net_c = lnr.lnr_unet_load(clean, blob, FP16)
    base_clean = lnr.lnr_allocated_bytes(clean)
    img = lnr.Image(H, W)
    (lnr.lnr_render_soft if soft else lnr.lnr_render)(clean, room_cloud, cam, img)
    lnr.lnr_depth_filter(clean, img, 4, 0.5)
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
    lnr.lnr_reconstruct(clean, net_c, img, out)
    lnr.lnr_sync(clean)
    scratch = lnr.lnr_allocated_bytes(clean) - base_clean

    ctx = lnr.lnr_context_create(0)
    net = lnr.lnr_unet_load(ctx, blob, FP16)
    base = lnr.lnr_allocated_bytes(ctx)
    img = _sentinel_image(lnr, H, W)
    render = (lambda: lnr.lnr_render_soft(ctx, room_cloud, cam, img)) if soft else \
        (lambda: lnr.lnr_render(ctx, room_cloud, cam, img))
    fails = 0
    for _ in _sweep(lnr, ctx, render):
        assert _untouched(img), "a failed render wrote the image"
        fails += 1
    # the context's scratch is grow-only and kept: after the n-th allocation
    # fails, the ones before it stay, so the next attempt starts further on
    # (hard: flags, work queues, counters -> 2 failing attempts; soft adds the
    # colour sums -> 3)
    assert fails >= (3 if soft else 2)
    fimg = _sentinel_image(lnr, H, W)
    fimg.key = None
    for _ in _sweep(lnr, ctx, lambda: lnr.lnr_depth_filter(ctx, fimg, 4, 0.5)):
        torch.cuda.synchronize()
        assert bool((fimg.depth == -3.25).all()) and bool((fimg.rgba == 0xA5).all())
    out = torch.full((3, H, W), 7.0, dtype=torch.float32, device="cuda")
    for _ in _sweep(lnr, ctx, lambda: lnr.lnr_reconstruct(ctx, net, img, out)):
        torch.cuda.synchronize()
        assert bool((out == 7.0).all()), "a failed reconstruct wrote the output"
    lnr.lnr_sync(ctx)
    # the failed attempts left no allocation beyond the scratch of a clean run
    assert lnr.lnr_allocated_bytes(ctx) - base == scratch


def test_server_create_and_sessions_free_everything_on_failure(lnr, room_cloud):
    ctx = lnr.lnr_context_create(0)
    net = lnr.lnr_unet_load(ctx, synth.make_unet_blob((16, 32, 64), seed=0), FP16)
    base = lnr.lnr_allocated_bytes(ctx)
    holder = []
    fails = 0
    for _ in _sweep(lnr, ctx, lambda: holder.append(lnr.lnr_server_create(
            ctx, room_cloud, net, max_batch=2, lanes=2, n_levels=3, max_width=128, max_height=96))):
        assert lnr.lnr_allocated_bytes(ctx) == base
        fails += 1
    assert fails >= 6
    srv = holder[-1]
    with_srv = lnr.lnr_allocated_bytes(ctx)
    for _ in _sweep(lnr, ctx, lambda: lnr.lnr_server_open_session(srv, 64, 48)):
        assert lnr.lnr_allocated_bytes(ctx) == with_srv
    lnr.lnr_server_destroy(srv)
    assert lnr.lnr_allocated_bytes(ctx) == base


def test_server_rejects_a_session_too_small_for_its_filter_levels(lnr, room_cloud):
    ctx = lnr.lnr_context_create(0)
    net = lnr.lnr_unet_load(ctx, synth.make_unet_blob((16, 32), seed=0), FP16)
    srv = lnr.lnr_server_create(ctx, room_cloud, net, max_batch=2, lanes=1, n_levels=5, max_width=128,
                                max_height=96)
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_server_open_session(srv, 64, 16)   # floor(log2(16)) = 4 < 5 levels
    assert e.value.status == lnr.LNR_E_INVALID_ARG
    sid = lnr.lnr_server_open_session(srv, 64, 32)
    assert sid >= 0
    assert lnr.lnr_server_pending(srv) == (0, 0)
    lnr.lnr_server_destroy(srv)


def test_unknown_precision_is_rejected(lnr, ctx):
    blob = synth.make_unet_blob((16, 32), seed=0)
    for prec in (6, 99, -1):
        with pytest.raises(lnr.LnrError) as e:
            lnr.lnr_unet_load(ctx, blob, prec)
        assert e.value.status == lnr.LNR_E_INVALID_ARG
    for prec in (lnr.LNR_FP8_E4M3, lnr.LNR_FP8_E4M3X3):
        lnr.lnr_unet_destroy(lnr.lnr_unet_load(ctx, blob, prec))


def test_render_views_leaves_outputs_untouched(lnr, room_cloud, room_cams):
    """Each allocation of a multi-view render in turn fails: no image is
    written, and the scratch left equals a clean run's."""
    cams = list(room_cams[:10])
    clean = lnr.lnr_context_create(0)
    lnr.lnr_render_views(clean, room_cloud, cams, [lnr.Image(c.height, c.width) for c in cams])
    lnr.lnr_sync(clean)
    scratch = lnr.lnr_allocated_bytes(clean)
    ctx = lnr.lnr_context_create(0)
    imgs = [_sentinel_image(lnr, c.height, c.width) for c in cams]
    fails = 0
    for _ in _sweep(lnr, ctx, lambda: lnr.lnr_render_views(ctx, room_cloud, cams, imgs)):
        assert all(_untouched(i) for i in imgs), "a failed multi-view render wrote an image"
        fails += 1
    # cull flags, work items and counters; the grow-only scratch keeps what
    # an attempt allocated before its failure, so the third attempt succeeds
    assert fails >= 2
    lnr.lnr_sync(ctx)
    assert lnr.lnr_allocated_bytes(ctx) == scratch
