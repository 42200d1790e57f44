"""ctypes binding of liblnr (include/lnr.h), same names as the C entry points.

Argument marshalling only: every stage runs in the library's HIP kernels.
Device buffers are torch tensors (their data_ptr is passed), host buffers are
numpy arrays, and the stream is a torch stream (default: the current one).
A failing call raises LnrError with the library's status and message.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblnr.so")

LNR_OK = 0
LNR_E_INVALID_ARG = -1
LNR_E_OUT_OF_MEMORY = -2
LNR_E_BUDGET = -3
LNR_E_DEVICE = -4
LNR_E_UNSUPPORTED = -5
LNR_E_FORMAT = -6

LNR_FP32 = 0
LNR_BF16 = 1
LNR_FP8_E4M3 = 2
LNR_BF16X3 = 3
LNR_FP16 = 4
LNR_FP8_E4M3X3 = 5

LNR_RENDER_NO_CULL = 1
LNR_RENDER_COUNT_ATOMICS = 2
LNR_RENDER_ATOMIC_SPLAT = 4

EMPTY_KEY = 0xFFFFFFFFFFFFFFFF


class LnrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lnr status {status}: {message}")
        self.status = status


class lnr_camera(ctypes.Structure):
    _fields_ = [("P", ctypes.c_float * 12), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_float), ("z_far", ctypes.c_float)]


class lnr_image(ctypes.Structure):
    _fields_ = [("key", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("rgba", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


class lnr_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("ms", ctypes.c_float)]


class lnr_server_config(ctypes.Structure):
    _fields_ = [("max_batch", ctypes.c_int32), ("lanes", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("filter_strength", ctypes.c_float), ("soft", ctypes.c_int32), ("soft_eps", ctypes.c_float),
                ("use_graphs", ctypes.c_int32), ("max_width", ctypes.c_int32), ("max_height", ctypes.c_int32)]


class lnr_server_result(ctypes.Structure):
    _fields_ = [("session", ctypes.c_int32), ("tag", ctypes.c_uint64), ("superseded", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("batch_gpu_ms", ctypes.c_float), ("rgb", ctypes.c_void_p),
                ("width", ctypes.c_int32), ("height", ctypes.c_int32)]


def _hip_runtimes():
    """Distinct HIP runtime libraries mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return paths


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2502_11618_amd.build` "
                          "(there is no fallback implementation)")
    # torch ships its own HIP runtime under the same soname; loading it first makes
    # liblnr.so bind to that same runtime, so torch's streams and device pointers
    # are valid in the library (two runtimes in one process do not share devices).
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    rt = _hip_runtimes()
    if len(rt) > 1:
        raise ImportError(f"more than one HIP runtime is loaded ({sorted(rt)}); import torch before liblnr.so")
    vp, u64, i32, f32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_float
    sig = {
        "lnr_context_create": (i32, [ctypes.c_int, u64, ctypes.POINTER(vp)]),
        "lnr_context_destroy": (None, [vp]),
        "lnr_last_error": (ctypes.c_char_p, [vp]),
        "lnr_allocated_bytes": (u64, [vp]),
        "lnr_cloud_load": (i32, [vp, vp, vp, u64, f32, ctypes.POINTER(vp)]),
        "lnr_cloud_info": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(i32 * 3), ctypes.POINTER(f32 * 3),
                                 ctypes.POINTER(f32)]),
        "lnr_cloud_permutation": (i32, [vp, vp]),
        "lnr_cloud_cell_start": (i32, [vp, vp]),
        "lnr_cloud_destroy": (None, [vp]),
        "lnr_render": (i32, [vp, vp, ctypes.POINTER(lnr_camera), ctypes.POINTER(lnr_image), ctypes.c_uint32, vp]),
        "lnr_render_soft": (i32, [vp, vp, ctypes.POINTER(lnr_camera), ctypes.POINTER(lnr_image), f32, ctypes.c_uint32,
                                  vp]),
        "lnr_render_views": (i32, [vp, vp, ctypes.POINTER(lnr_camera), ctypes.POINTER(lnr_image), i32,
                                   ctypes.c_uint32, vp]),
        "lnr_render_stats": (i32, [vp, ctypes.POINTER(u64), ctypes.POINTER(u64), vp]),
        "lnr_render_atomic_count": (i32, [vp, ctypes.POINTER(u64)]),
        "lnr_measure_atomic_min": (i32, [vp, u64, i32, u64, vp, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(u64)]),
        "lnr_depth_filter": (i32, [vp, ctypes.POINTER(lnr_image), i32, f32, vp]),
        "lnr_depth_filter_noalloc": (i32, [vp, ctypes.POINTER(lnr_image), i32, f32, vp]),
        "lnr_unet_load": (i32, [vp, vp, u64, ctypes.c_int, ctypes.POINTER(vp)]),
        "lnr_unet_destroy": (None, [vp]),
        "lnr_reconstruct": (i32, [vp, vp, ctypes.POINTER(lnr_image), vp, vp]),
        "lnr_sync": (i32, [vp, vp]),
        "lnr_profile_enable": (i32, [vp, ctypes.c_int]),
        "lnr_debug_fail_allocation": (i32, [vp, ctypes.c_int64]),
        "lnr_profile_read": (i32, [vp, ctypes.POINTER(lnr_kernel_time), i32, ctypes.POINTER(i32)]),
        "lnr_server_create": (i32, [vp, vp, vp, ctypes.POINTER(lnr_server_config), ctypes.POINTER(vp)]),
        "lnr_server_destroy": (None, [vp]),
        "lnr_server_open_session": (i32, [vp, i32, i32, ctypes.POINTER(i32)]),
        "lnr_server_close_session": (i32, [vp, i32]),
        "lnr_server_submit": (i32, [vp, i32, ctypes.POINTER(lnr_camera), u64]),
        "lnr_server_step": (i32, [vp, ctypes.POINTER(i32)]),
        "lnr_server_poll": (i32, [vp, ctypes.POINTER(lnr_server_result), i32, ctypes.POINTER(i32)]),
        "lnr_server_pending": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
lib = _lib


def _check(st: int, ctx) -> None:
    if st != LNR_OK:
        msg = _lib.lnr_last_error(ctx)
        raise LnrError(st, msg.decode() if msg else "")


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


# ---------------------------------------------------------------------------
# handles
# ---------------------------------------------------------------------------

class Cloud:
    def __init__(self, ctx, handle):
        self.ctx = ctx
        self.handle = handle

    def info(self):
        return lnr_cloud_info(self)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnr_cloud_destroy(self.handle)
            self.handle = None


class UNet:
    def __init__(self, ctx, handle, prec, widths):
        self.ctx = ctx
        self.handle = handle
        self.precision = prec
        self.widths = widths

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnr_unet_destroy(self.handle)
            self.handle = None


class Context:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnr_context_destroy(self.handle)
            self.handle = None


class Image:
    """RGBDA image in device memory (torch tensors): key int64 [H*W] (the
    uint64 key bits), depth float32 [H, W], rgba uint8 [H, W, 4]."""

    def __init__(self, height: int, width: int, device="cuda", with_key: bool = True):
        import torch
        self.height, self.width = int(height), int(width)
        n = self.height * self.width
        self.key = torch.empty(n, dtype=torch.int64, device=device) if with_key else None
        self.depth = torch.empty((self.height, self.width), dtype=torch.float32, device=device)
        self.rgba = torch.empty((self.height, self.width, 4), dtype=torch.uint8, device=device)

    @classmethod
    def from_tensors(cls, depth, rgba, key=None):
        img = cls.__new__(cls)
        img.height, img.width = int(depth.shape[0]), int(depth.shape[1])
        img.depth, img.rgba, img.key = depth, rgba, key
        return img

    def struct(self) -> lnr_image:
        return lnr_image(_ptr(self.key), _ptr(self.depth), _ptr(self.rgba), self.width, self.height)


def camera_struct(cam) -> lnr_camera:
    c = lnr_camera()
    P = np.asarray(cam.P, dtype=np.float32)
    for i in range(12):
        c.P[i] = float(P[i])
    c.width, c.height = int(cam.width), int(cam.height)
    c.z_near, c.z_far = float(np.float32(cam.z_near)), float(np.float32(cam.z_far))
    return c


# ---------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ---------------------------------------------------------------------------

def lnr_context_create(hip_device: int = 0, hbm_budget_bytes: int = 0) -> Context:
    h = ctypes.c_void_p()
    _check(_lib.lnr_context_create(hip_device, hbm_budget_bytes, ctypes.byref(h)), None)
    return Context(h.value)


def lnr_context_destroy(ctx: Context) -> None:
    """Frees the context and its scratch.  Clouds, networks and servers
    created through it must be destroyed first."""
    ctx.__del__()


def lnr_last_error(ctx: Optional[Context]) -> str:
    msg = _lib.lnr_last_error(ctx.handle if ctx is not None else None)
    return msg.decode() if msg else ""


def lnr_allocated_bytes(ctx: Context) -> int:
    return int(_lib.lnr_allocated_bytes(ctx.handle))


def lnr_cloud_load(ctx: Context, xyz: np.ndarray, rgb: np.ndarray, cell_size: float) -> Cloud:
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    rgb = np.ascontiguousarray(rgb, dtype=np.uint8)
    if xyz.ndim != 2 or xyz.shape[1] != 3 or rgb.shape != xyz.shape:
        raise ValueError("xyz must be float32 [n, 3] and rgb uint8 [n, 3]")
    h = ctypes.c_void_p()
    _check(_lib.lnr_cloud_load(ctx.handle, xyz.ctypes.data, rgb.ctypes.data, xyz.shape[0], float(cell_size),
                               ctypes.byref(h)), ctx.handle)
    return Cloud(ctx, h.value)


def lnr_cloud_destroy(cloud: Cloud) -> None:
    cloud.__del__()


def lnr_cloud_info(cloud: Cloud):
    n = ctypes.c_uint64()
    dims = (ctypes.c_int32 * 3)()
    origin = (ctypes.c_float * 3)()
    s = ctypes.c_float()
    _check(_lib.lnr_cloud_info(cloud.handle, ctypes.byref(n), ctypes.byref(dims), ctypes.byref(origin),
                               ctypes.byref(s)), cloud.ctx.handle)
    return dict(n=n.value, dims=tuple(dims), origin=np.array(origin[:], np.float32), cell_size=s.value)


def lnr_cloud_permutation(cloud: Cloud) -> np.ndarray:
    n = lnr_cloud_info(cloud)["n"]
    out = np.empty(n, dtype=np.uint32)
    _check(_lib.lnr_cloud_permutation(cloud.handle, out.ctypes.data), cloud.ctx.handle)
    return out


def lnr_cloud_cell_start(cloud: Cloud) -> np.ndarray:
    d = lnr_cloud_info(cloud)["dims"]
    out = np.empty(d[0] * d[1] * d[2] + 1, dtype=np.uint32)
    _check(_lib.lnr_cloud_cell_start(cloud.handle, out.ctypes.data), cloud.ctx.handle)
    return out


def lnr_render(ctx: Context, cloud: Cloud, cam, image: Image, flags: int = 0, stream=None) -> None:
    c = cam if isinstance(cam, lnr_camera) else camera_struct(cam)
    img = image.struct()
    _check(_lib.lnr_render(ctx.handle, cloud.handle, ctypes.byref(c), ctypes.byref(img), flags, _stream(stream)),
           ctx.handle)


def lnr_render_soft(ctx: Context, cloud: Cloud, cam, image: Image, soft_eps: float = 0.01, flags: int = 0,
                    stream=None) -> None:
    c = cam if isinstance(cam, lnr_camera) else camera_struct(cam)
    img = image.struct()
    _check(_lib.lnr_render_soft(ctx.handle, cloud.handle, ctypes.byref(c), ctypes.byref(img), float(soft_eps), flags,
                                _stream(stream)), ctx.handle)


def lnr_render_views(ctx: Context, cloud: Cloud, cams, images, flags: int = 0, stream=None) -> None:
    """Several views in one pass over the cloud; cams and images are sequences
    of equal length (images[v] receives what lnr_render of cams[v] writes)."""
    n = len(cams)
    c_arr = (lnr_camera * max(n, 1))(*[c if isinstance(c, lnr_camera) else camera_struct(c) for c in cams])
    i_arr = (lnr_image * max(len(images), 1))(*[im.struct() for im in images])
    _check(_lib.lnr_render_views(ctx.handle, cloud.handle, c_arr, i_arr, n, flags, _stream(stream)), ctx.handle)


def lnr_render_stats(ctx: Context, n_cells: Optional[int] = None):
    vis = ctypes.c_uint64()
    proc = ctypes.c_uint64()
    flags = np.empty(n_cells, dtype=np.uint8) if n_cells else None
    _check(_lib.lnr_render_stats(ctx.handle, ctypes.byref(vis), ctypes.byref(proc),
                                 flags.ctypes.data if flags is not None else None), ctx.handle)
    return vis.value, proc.value, flags


def lnr_render_atomic_count(ctx: Context) -> int:
    n = ctypes.c_uint64()
    _check(_lib.lnr_render_atomic_count(ctx.handle, ctypes.byref(n)), ctx.handle)
    return n.value


def lnr_measure_atomic_min(ctx: Context, n_slots: int, pattern: int, n_ops: int, stream=None):
    """(operations per second, operations timed)"""
    rate = ctypes.c_double()
    done = ctypes.c_uint64()
    _check(_lib.lnr_measure_atomic_min(ctx.handle, int(n_slots), int(pattern), int(n_ops), _stream(stream),
                                       ctypes.byref(rate), ctypes.byref(done)), ctx.handle)
    return rate.value, done.value


def lnr_depth_filter(ctx: Context, image: Image, n_levels: int, filter_strength: float, stream=None) -> None:
    img = image.struct()
    _check(_lib.lnr_depth_filter(ctx.handle, ctypes.byref(img), int(n_levels), float(filter_strength),
                                 _stream(stream)), ctx.handle)


def lnr_depth_filter_noalloc(ctx: Context, image: Image, n_levels: int, filter_strength: float, stream=None) -> None:
    img = image.struct()
    _check(_lib.lnr_depth_filter_noalloc(ctx.handle, ctypes.byref(img), int(n_levels), float(filter_strength),
                                         _stream(stream)), ctx.handle)


def lnr_unet_load(ctx: Context, blob: bytes, precision: int = LNR_FP32) -> UNet:
    import struct
    buf = ctypes.create_string_buffer(bytes(blob), len(blob))
    h = ctypes.c_void_p()
    _check(_lib.lnr_unet_load(ctx.handle, ctypes.addressof(buf), len(blob), int(precision), ctypes.byref(h)),
           ctx.handle)
    L = struct.unpack_from("<I", blob, 8)[0]
    widths = struct.unpack_from(f"<{L}I", blob, 20)
    return UNet(ctx, h.value, precision, widths)


def lnr_unet_destroy(unet: UNet) -> None:
    unet.__del__()


def lnr_reconstruct(ctx: Context, unet: UNet, image: Image, rgb_out, stream=None) -> None:
    img = image.struct()
    _check(_lib.lnr_reconstruct(ctx.handle, unet.handle, ctypes.byref(img), rgb_out.data_ptr(), _stream(stream)),
           ctx.handle)


def lnr_sync(ctx: Context, stream=None) -> None:
    _check(_lib.lnr_sync(ctx.handle, _stream(stream)), ctx.handle)


def lnr_profile_enable(ctx: Context, enable: bool = True) -> None:
    _check(_lib.lnr_profile_enable(ctx.handle, 1 if enable else 0), ctx.handle)


def lnr_debug_fail_allocation(ctx: Context, after: int) -> None:
    """Make the device allocation after `after` successful ones fail (-1: off)."""
    _check(_lib.lnr_debug_fail_allocation(ctx.handle, int(after)), ctx.handle)


def lnr_profile_read(ctx: Context, max_records: int = 1 << 16):
    """[(name, ms)] of the launches timed since the last read, oldest first."""
    buf = (lnr_kernel_time * max_records)()
    n = ctypes.c_int32()
    _check(_lib.lnr_profile_read(ctx.handle, buf, max_records, ctypes.byref(n)), ctx.handle)
    return [(buf[i].name.decode(), float(buf[i].ms)) for i in range(min(n.value, max_records))]


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

class Server:
    def __init__(self, ctx, handle, keep):
        self.ctx = ctx
        self.handle = handle
        self._keep = keep  # the cloud and network must outlive the server

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.lnr_server_destroy(self.handle)
            self.handle = None


def lnr_server_create(ctx: Context, cloud: Cloud, unet: UNet, max_batch: int = 8, lanes: int = 2,
                      n_levels: int = 5, filter_strength: float = 0.5, soft: bool = False, soft_eps: float = 0.01,
                      use_graphs: bool = True, max_width: int = 1920, max_height: int = 1080) -> Server:
    cfg = lnr_server_config(max_batch, lanes, n_levels, filter_strength, 1 if soft else 0, soft_eps,
                            1 if use_graphs else 0, max_width, max_height)
    h = ctypes.c_void_p()
    _check(_lib.lnr_server_create(ctx.handle, cloud.handle, unet.handle, ctypes.byref(cfg), ctypes.byref(h)),
           ctx.handle)
    return Server(ctx, h.value, (cloud, unet))


def lnr_server_destroy(srv: Server) -> None:
    """Waits for the server's in-flight batches and frees its lanes and sessions."""
    srv.__del__()


def lnr_server_open_session(srv: Server, width: int, height: int) -> int:
    sid = ctypes.c_int32()
    _check(_lib.lnr_server_open_session(srv.handle, int(width), int(height), ctypes.byref(sid)), srv.ctx.handle)
    return sid.value


def lnr_server_close_session(srv: Server, session: int) -> None:
    _check(_lib.lnr_server_close_session(srv.handle, int(session)), srv.ctx.handle)


def lnr_server_submit(srv: Server, session: int, cam, tag: int) -> None:
    c = cam if isinstance(cam, lnr_camera) else camera_struct(cam)
    _check(_lib.lnr_server_submit(srv.handle, int(session), ctypes.byref(c), int(tag)), srv.ctx.handle)


def lnr_server_step(srv: Server) -> int:
    n = ctypes.c_int32()
    _check(_lib.lnr_server_step(srv.handle, ctypes.byref(n)), srv.ctx.handle)
    return n.value


def lnr_server_poll(srv: Server, max_results: int = 1024):
    buf = (lnr_server_result * max_results)()
    n = ctypes.c_int32()
    _check(_lib.lnr_server_poll(srv.handle, buf, max_results, ctypes.byref(n)), srv.ctx.handle)
    return [dict(session=r.session, tag=r.tag, superseded=bool(r.superseded), batch=r.batch,
                 batch_gpu_ms=r.batch_gpu_ms, rgb=r.rgb, width=r.width, height=r.height) for r in buf[:n.value]]


def lnr_server_pending(srv: Server):
    p = ctypes.c_int32()
    f = ctypes.c_int32()
    _check(_lib.lnr_server_pending(srv.handle, ctypes.byref(p), ctypes.byref(f)), srv.ctx.handle)
    return p.value, f.value


def copy_from_device(ptr: int, out) -> None:
    """Copy out.numel() elements from library-owned device memory at `ptr` into
    the torch tensor `out` (hipMemcpy of the HIP runtime the library shares
    with torch)."""
    global _hip
    if _hip is None:
        (path,) = _hip_runtimes()
        _hip = ctypes.CDLL(path)
        _hip.hipMemcpy.restype = ctypes.c_int
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    err = _hip.hipMemcpy(out.data_ptr(), ptr, out.numel() * out.element_size(), 3)  # device to device
    if err != 0:
        raise LnrError(LNR_E_DEVICE, f"hipMemcpy failed ({err})")


_hip = None
