"""The serving loop: every session's frame computed in a batch of mixed
sessions equals the same frame computed alone; admission by budget; newer
cameras supersede pending ones."""

import numpy as np
import pytest

import synth
from oracle import depth_filter as F
from oracle import metrics as M
from oracle import render as R
from oracle import unet as U
from tests.gpu_util import render_gpu

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (128, 96), (64, 64), (128, 96), (64, 64), (96, 64), (64, 64)]


def _alone(lnr, ctx, cloud, net, cam, n_levels, fs):
    import torch
    img = render_gpu(lnr, ctx, cloud, cam)
    if n_levels:
        lnr.lnr_depth_filter(ctx, img, n_levels, fs)
    out = torch.empty((3, cam.height, cam.width), dtype=torch.float32, device="cuda")
    lnr.lnr_reconstruct(ctx, net, img, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _serve_all(lnr, srv, sids, cams_per_session, frames):
    import torch
    results = {}
    for f in range(frames):
        for i, sid in enumerate(sids):
            lnr.lnr_server_submit(srv, sid, cams_per_session[i][f], tag=f * 100 + i)
        got = 0
        for _ in range(100000):
            lnr.lnr_server_step(srv)
            for r in lnr.lnr_server_poll(srv):
                assert not r["superseded"]
                out = torch.empty((3, r["height"], r["width"]), dtype=torch.float32, device="cuda")
                lnr.copy_from_device(r["rgb"], out)
                results[r["tag"]] = (out.cpu().numpy(), r["batch"])
                got += 1
            if got == len(sids):
                break
        assert got == len(sids), "server did not finish"
    return results


@pytest.mark.parametrize("prec,graphs", [(0, True), (1, True), (3, False), (4, True), (5, True), (2, False)])
def test_mixed_batches_equal_alone(lnr, ctx, room_scene, room_cloud, room_grid, prec, graphs):
    blob = synth.make_unet_blob((16, 32, 64), seed=0)
    net = lnr.lnr_unet_load(ctx, blob, prec)
    srv = lnr.lnr_server_create(ctx, room_cloud, net, max_batch=4, lanes=2, n_levels=3, filter_strength=0.5,
                                use_graphs=graphs, max_width=128, max_height=96)
    sids = [lnr.lnr_server_open_session(srv, w, h) for (w, h) in SIZES]
    cams = [synth.random_walk_path(room_scene, 3, seed=i, width=w, height=h, fov_deg=80.0)
            for i, (w, h) in enumerate(SIZES)]
    res = _serve_all(lnr, srv, sids, cams, 3)
    assert max(b for _, b in res.values()) > 1, "no batch had more than one request"
    onet = U.parse_blob(blob)
    for f in range(3):
        for i in range(len(SIZES)):
            got, _ = res[f * 100 + i]
            cam = cams[i][f]
            alone = _alone(lnr, ctx, room_cloud, net, cam, 3, 0.5)
            assert np.array_equal(got, alone), f"session {i} frame {f} differs from its standalone render"
            if f == 0 and prec == 0:
                _, depth, rgba = R.render(room_grid, cam)
                fd, fr, _ = F.depth_filter(depth.reshape(cam.height, cam.width),
                                           rgba.reshape(cam.height, cam.width, 4), 3, 0.5)
                assert M.max_abs(got, U.forward(onet, fd, fr)) <= 1e-4


def test_superseded_requests_and_admission(lnr, room_scene, room_cloud):
    ctx = lnr.lnr_context_create(0)
    blob = synth.make_unet_blob((16, 32, 64), seed=0)
    net = lnr.lnr_unet_load(ctx, blob, lnr.LNR_BF16)
    cloud = lnr.lnr_cloud_load(ctx, room_scene.xyz, room_scene.rgb, 0.5)
    srv = lnr.lnr_server_create(ctx, cloud, net, max_batch=2, lanes=1, n_levels=3, max_width=64, max_height=64)
    sid = lnr.lnr_server_open_session(srv, 64, 64)
    cams = synth.random_walk_path(room_scene, 2, seed=1, width=64, height=64)
    lnr.lnr_server_submit(srv, sid, cams[0], tag=1)
    lnr.lnr_server_submit(srv, sid, cams[1], tag=2)   # replaces tag 1 before it runs
    seen = {}
    for _ in range(100000):
        lnr.lnr_server_step(srv)
        for r in lnr.lnr_server_poll(srv):
            seen[r["tag"]] = r["superseded"]
        if 2 in seen:
            break
    assert seen == {1: True, 2: False}
    # admission by budget: measure what a server and one session need on an
    # unlimited context, then give a fresh context room for exactly two sessions
    big = lnr.lnr_context_create(0)
    net_b = lnr.lnr_unet_load(big, blob, lnr.LNR_BF16)
    srv_b = lnr.lnr_server_create(big, cloud, net_b, max_batch=2, lanes=1, n_levels=3, max_width=64, max_height=64)
    base = lnr.lnr_allocated_bytes(big)
    lnr.lnr_server_open_session(srv_b, 64, 64)
    per_session = lnr.lnr_allocated_bytes(big) - base
    small = lnr.lnr_context_create(0, base + int(2.5 * per_session))
    net_s = lnr.lnr_unet_load(small, blob, lnr.LNR_BF16)
    srv_s = lnr.lnr_server_create(small, cloud, net_s, max_batch=2, lanes=1, n_levels=3, max_width=64,
                                  max_height=64)
    assert lnr.lnr_allocated_bytes(small) == base
    lnr.lnr_server_open_session(srv_s, 64, 64)
    lnr.lnr_server_open_session(srv_s, 64, 64)
    with pytest.raises(lnr.LnrError) as e:
        lnr.lnr_server_open_session(srv_s, 64, 64)
    assert e.value.status == lnr.LNR_E_BUDGET


def test_soft_zbuffer_sessions_equal_alone(lnr, ctx, room_scene, room_cloud):
    """Serving with the soft z-buffer: every frame equals lnr_render_soft +
    filter + reconstruct of the same camera."""
    import torch
    blob = synth.make_unet_blob((16, 32, 64), seed=1)
    net = lnr.lnr_unet_load(ctx, blob, lnr.LNR_FP32)
    srv = lnr.lnr_server_create(ctx, room_cloud, net, max_batch=4, lanes=2, n_levels=3, filter_strength=0.5,
                                soft=True, soft_eps=0.02, use_graphs=True, max_width=128, max_height=96)
    sizes = [(128, 96), (64, 64), (128, 96)]
    sids = [lnr.lnr_server_open_session(srv, w, h) for (w, h) in sizes]
    cams = [synth.random_walk_path(room_scene, 2, seed=30 + i, width=w, height=h, fov_deg=80.0)
            for i, (w, h) in enumerate(sizes)]
    res = _serve_all(lnr, srv, sids, cams, 2)
    for f in range(2):
        for i, (w, h) in enumerate(sizes):
            cam = cams[i][f]
            img = lnr.Image(h, w)
            lnr.lnr_render_soft(ctx, room_cloud, cam, img, 0.02)
            lnr.lnr_depth_filter(ctx, img, 3, 0.5)
            out = torch.empty((3, h, w), dtype=torch.float32, device="cuda")
            lnr.lnr_reconstruct(ctx, net, img, out)
            torch.cuda.synchronize()
            assert np.array_equal(res[f * 100 + i][0], out.cpu().numpy()), f"session {i} frame {f}"


@pytest.mark.parametrize("prec", [0, 1])
def test_two_context_frame_pipeline_equals_sequential(lnr, ctx, room_cloud, room_cams, prec):
    """The frame pipeline the bench times: projection and filter of frame i on
    one stream and context while the U-Net of frame i - 1 runs on another,
    two RGBDA images alternating.  Every frame's output equals the frame
    computed alone on one stream, bit for bit."""
    import torch
    W = H = 256
    net = lnr.lnr_unet_load(ctx, synth.make_unet_blob((16, 32, 64), seed=3), prec)
    ctx_geo = lnr.lnr_context_create(0)
    alone = []
    img = lnr.Image(H, W)
    for cam in room_cams[:6]:
        lnr.lnr_render(ctx, room_cloud, cam, img)
        lnr.lnr_depth_filter(ctx, img, 4, 0.5)
        o = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
        lnr.lnr_reconstruct(ctx, net, img, o)
        alone.append(o)
    torch.cuda.synchronize()
    s_geo, s_net = torch.cuda.Stream(), torch.cuda.current_stream()
    imgs = [lnr.Image(H, W), lnr.Image(H, W)]
    ready = [torch.cuda.Event(), torch.cuda.Event()]
    done = [torch.cuda.Event(), torch.cuda.Event()]
    for e in done:
        e.record(s_net)
    outs = []
    for i, cam in enumerate(room_cams[:6]):
        g = i & 1
        s_geo.wait_event(done[g])
        lnr.lnr_render(ctx_geo, room_cloud, cam, imgs[g], stream=s_geo)
        lnr.lnr_depth_filter(ctx_geo, imgs[g], 4, 0.5, stream=s_geo)
        ready[g].record(s_geo)
        s_net.wait_event(ready[g])
        o = torch.empty((3, H, W), dtype=torch.float32, device="cuda")
        lnr.lnr_reconstruct(ctx, net, imgs[g], o, stream=s_net)
        done[g].record(s_net)
        outs.append(o)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(alone, outs)):
        assert torch.equal(a, b), f"frame {i} differs in the pipeline"


def test_whole_batch_graph_replays_follow_new_cameras(lnr, ctx, room_scene, room_cloud):
    """One lane, two sessions of one size: every step replays the one captured
    graph of (96 x 128, batch 2) with the next cameras, written to device
    memory before the replay.  Each of 6 replays, with the checks' own device
    work in between, must equal the frames computed alone."""
    blob = synth.make_unet_blob((16, 32, 64), seed=2)
    net = lnr.lnr_unet_load(ctx, blob, lnr.LNR_FP32)
    srv = lnr.lnr_server_create(ctx, room_cloud, net, max_batch=2, lanes=1, n_levels=3, filter_strength=0.5,
                                use_graphs=True, max_width=128, max_height=96)
    sids = [lnr.lnr_server_open_session(srv, 128, 96) for _ in range(2)]
    cams = [synth.random_walk_path(room_scene, 6, seed=50 + i, width=128, height=96, fov_deg=80.0) for i in range(2)]
    res = _serve_all(lnr, srv, sids, cams, 6)
    assert all(b == 2 for _, b in res.values())
    for f in range(6):
        for i in range(2):
            alone = _alone(lnr, ctx, room_cloud, net, cams[i][f], 3, 0.5)
            assert np.array_equal(res[f * 100 + i][0], alone), f"session {i} frame {f}"
