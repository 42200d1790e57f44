"""Synthetic static-LiDAR scenes.

The paper evaluates on indoor multi-scan LiDAR clouds of about 23M points and
names three artefacts of such scans (Introduction): incomplete coverage /
occlusion gaps, colour inconsistencies between scans, and density that falls
off with distance from the scanner.  The generators below reproduce those
three properties from a seed; no dataset item is reproduced.

Scanner model: each scan casts rays with directions uniform on the unit
sphere from one scanner position; every ray is intersected analytically with
the scene (axis-aligned rectangles, spheres, axis-aligned boxes, vertical
cylinders) and the nearest hit beyond 5 cm becomes a point.  Uniform
solid-angle sampling gives a surface density proportional to cos(theta)/r^2.
Colours are an integer base colour per surface plus N(0, 8) noise per
channel, times a per-scan, per-channel gain N(1, 0.05) (multi-scan scenes
only), rounded to nearest and clipped to uint8.  Multi-scan scenes also drop
rays inside random spherical caps (angular radius 5-20 degrees) until 20% of
each scan's directions are covered, and keep casting until the scan's quota
is met.
"""

from __future__ import annotations

import dataclasses
import hashlib
import os
from concurrent.futures import ProcessPoolExecutor
from typing import Callable, List, Optional, Tuple

import numpy as np

T_MIN = 0.05  # nearest accepted hit distance along a ray (m)


@dataclasses.dataclass
class Primitives:
    # axis-aligned rectangles: axis, c, lo1, hi1, lo2, hi2, surface id
    rects: np.ndarray
    # spheres: cx, cy, cz, r, surface id
    spheres: np.ndarray
    # solid boxes: x0, y0, z0, x1, y1, z1, surface id
    boxes: np.ndarray
    # vertical cylinders: cx, cy, r, z0, z1, surface id
    cylinders: np.ndarray
    # base colours per surface id, uint8 [S, 3]
    colors: np.ndarray


@dataclasses.dataclass
class Scene:
    xyz: np.ndarray          # float32 [N, 3], interleaved, in ray order
    rgb: np.ndarray          # uint8 [N, 3]
    scanners: np.ndarray     # float64 [S, 3]
    bounds: Tuple[Tuple[float, float, float], Tuple[float, float, float]]
    room_centers: np.ndarray  # float64 [R, 3] centres of the rooms (z = 1.6)
    scanner_rooms: np.ndarray  # int [S] index of the room of each scanner
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


# ---------------------------------------------------------------------------
# ray / primitive intersection (float64, vectorised over rays of one origin)
# ---------------------------------------------------------------------------

def _hit_rects(s, d, rects, t_best, id_best):
    # rectangles sharing a plane share one ray/plane intersection
    with np.errstate(divide="ignore", invalid="ignore"):
        planes = {}
        for r in rects:
            planes.setdefault((int(r[0]), float(r[1])), []).append(r)
        for (axis, c), group in planes.items():
            a1, a2 = [a for a in range(3) if a != axis]
            t = (c - s[axis]) / d[:, axis]
            idx = np.nonzero((t > T_MIN) & (t < t_best))[0]
            if idx.size == 0:
                continue
            t = t[idx]
            p1 = s[a1] + t * d[idx, a1]
            p2 = s[a2] + t * d[idx, a2]
            for _, _, lo1, hi1, lo2, hi2, sid in group:
                ok = (p1 >= lo1) & (p1 <= hi1) & (p2 >= lo2) & (p2 <= hi2)
                sel = idx[ok]
                t_best[sel] = t[ok]
                id_best[sel] = int(sid)


def _cone_candidates(s, d, center, radius):
    """Indices of rays whose direction lies within the cone from s that bounds
    the sphere (center, radius); all rays when s is inside the sphere."""
    oc = np.asarray(center, dtype=np.float64) - s
    dist = float(np.sqrt(oc @ oc))
    if dist <= radius * 1.001:
        return np.arange(d.shape[0])
    cos_a = np.sqrt(max(0.0, 1.0 - (radius / dist) ** 2)) - 1e-9
    return np.nonzero(d @ (oc / dist) > cos_a)[0]


def _hit_spheres(s, d, spheres, t_best, id_best):
    for cx, cy, cz, r, sid in spheres:
        idx = _cone_candidates(s, d, (cx, cy, cz), r)
        if idx.size == 0:
            continue
        dd = d[idx]
        oc = s - np.array([cx, cy, cz])
        b = dd @ oc
        c = oc @ oc - r * r
        disc = b * b - c
        ok = disc >= 0
        t = -b - np.sqrt(np.where(ok, disc, 0.0))
        ok &= (t > T_MIN) & (t < t_best[idx])
        sel = idx[ok]
        t_best[sel] = t[ok]
        id_best[sel] = int(sid)


def _hit_boxes(s, d, boxes, t_best, id_best):
    with np.errstate(divide="ignore", invalid="ignore"):
        for x0, y0, z0, x1, y1, z1, sid in boxes:
            lo = np.array([x0, y0, z0])
            hi = np.array([x1, y1, z1])
            idx = _cone_candidates(s, d, 0.5 * (lo + hi), 0.5 * float(np.linalg.norm(hi - lo)))
            if idx.size == 0:
                continue
            inv = 1.0 / d[idx]
            t1 = (lo - s) * inv
            t2 = (hi - s) * inv
            tn = np.minimum(t1, t2).max(axis=1)
            tf = np.maximum(t1, t2).min(axis=1)
            ok = (tn <= tf) & (tn > T_MIN) & (tn < t_best[idx])
            sel = idx[ok]
            t_best[sel] = tn[ok]
            id_best[sel] = int(sid)


def _hit_cylinders(s, d, cyls, t_best, id_best):
    with np.errstate(divide="ignore", invalid="ignore"):
        for cx, cy, r, z0, z1, sid in cyls:
            center = (cx, cy, 0.5 * (z0 + z1))
            idx = _cone_candidates(s, d, center, float(np.hypot(r, 0.5 * (z1 - z0))))
            if idx.size == 0:
                continue
            dd = d[idx]
            ox, oy = s[0] - cx, s[1] - cy
            A = dd[:, 0] ** 2 + dd[:, 1] ** 2
            B = 2.0 * (ox * dd[:, 0] + oy * dd[:, 1])
            C = ox * ox + oy * oy - r * r
            disc = B * B - 4.0 * A * C
            ok = (disc >= 0) & (A > 0)
            t = (-B - np.sqrt(np.where(ok, disc, 0.0))) / (2.0 * A)
            z = s[2] + t * dd[:, 2]
            tb = t_best[idx]
            ok &= (t > T_MIN) & (t < tb) & (z >= z0) & (z <= z1)
            tb = np.where(ok, t, tb)
            hit = ok.copy()
            # top cap
            t = (z1 - s[2]) / dd[:, 2]
            px = s[0] + t * dd[:, 0] - cx
            py = s[1] + t * dd[:, 1] - cy
            ok = (t > T_MIN) & (t < tb) & (px * px + py * py <= r * r)
            tb = np.where(ok, t, tb)
            hit |= ok
            sel = idx[hit]
            t_best[sel] = tb[hit]
            id_best[sel] = int(sid)


def _cast(s: np.ndarray, d: np.ndarray, prims: Primitives):
    n = d.shape[0]
    t_best = np.full(n, np.inf)
    id_best = np.full(n, -1, dtype=np.int64)
    _hit_rects(s, d, prims.rects, t_best, id_best)
    _hit_spheres(s, d, prims.spheres, t_best, id_best)
    _hit_boxes(s, d, prims.boxes, t_best, id_best)
    _hit_cylinders(s, d, prims.cylinders, t_best, id_best)
    return t_best, id_best


def _uniform_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    rxy = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([rxy * np.cos(phi), rxy * np.sin(phi), z], axis=1)


def _make_caps(rng: np.random.Generator, coverage: float) -> np.ndarray:
    """Random spherical caps (unit centre, cos(radius)) covering `coverage` of the sphere."""
    caps: List[np.ndarray] = []
    probe = _uniform_dirs(rng, 200_000)
    covered = np.zeros(probe.shape[0], dtype=bool)
    while coverage > 0 and covered.mean() < coverage:
        c = _uniform_dirs(rng, 1)[0]
        rad = np.deg2rad(rng.uniform(5.0, 20.0))
        caps.append(np.array([c[0], c[1], c[2], np.cos(rad)]))
        covered |= probe @ c > np.cos(rad)
    return np.array(caps).reshape(-1, 4)


def _scan_chunk(args):
    (seed, scan_idx, chunk_idx, n_rays, s, prims, caps, gain) = args
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1 + scan_idx, chunk_idx])))
    d = _uniform_dirs(rng, n_rays)
    if caps.shape[0]:
        inside = np.zeros(n_rays, dtype=bool)
        for cap in caps:
            inside |= d @ cap[:3] > cap[3]
        d = d[~inside]
    t, sid = _cast(s, d, prims)
    ok = np.isfinite(t) & (sid >= 0)
    d, t, sid = d[ok], t[ok], sid[ok]
    pts = (s[None, :] + t[:, None] * d).astype(np.float32)
    base = prims.colors[sid].astype(np.float64)
    col = base + rng.normal(0.0, 8.0, size=base.shape)
    col = col * gain[None, :]
    rgb = np.clip(np.rint(col), 0, 255).astype(np.uint8)
    return pts, rgb


def _run_scans(seed, scanners, quota, prims, caps_list, gains, chunk_rays, workers):
    xyz_parts, rgb_parts = [], []
    for si, s in enumerate(scanners):
        need = quota
        chunk = 0
        got_xyz, got_rgb = [], []
        while need > 0:
            batch = []
            # enough chunks in flight to probably meet the quota in one round
            k = max(1, min(workers * 2, int(np.ceil(need / (0.75 * chunk_rays))) + 1))
            for j in range(k):
                batch.append((seed, si, chunk + j, chunk_rays, s, prims, caps_list[si], gains[si]))
            chunk += k
            if workers > 1 and k > 1:
                with ProcessPoolExecutor(max_workers=min(workers, k)) as ex:
                    results = list(ex.map(_scan_chunk, batch))
            else:
                results = [_scan_chunk(b) for b in batch]
            for p, c in results:
                if need <= 0:
                    break
                take = min(need, p.shape[0])
                got_xyz.append(p[:take])
                got_rgb.append(c[:take])
                need -= take
        xyz_parts.append(np.concatenate(got_xyz))
        rgb_parts.append(np.concatenate(got_rgb))
    return np.concatenate(xyz_parts), np.concatenate(rgb_parts)


def _default_workers() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


# ---------------------------------------------------------------------------
# scene layouts
# ---------------------------------------------------------------------------

def _box_walls(x1, y1, z1, first_sid):
    """The 6 inner faces of [0,x1]x[0,y1]x[0,z1]."""
    r = []
    sid = first_sid
    for c in (0.0, x1):
        r.append((0, c, 0.0, y1, 0.0, z1, sid)); sid += 1
    for c in (0.0, y1):
        r.append((1, c, 0.0, x1, 0.0, z1, sid)); sid += 1
    for c in (0.0, z1):
        r.append((2, c, 0.0, x1, 0.0, y1, sid)); sid += 1
    return r, sid


def room_scene(seed: int = 0, n_points: int = 200_000, workers: Optional[int] = None) -> Scene:
    """Small single-scan scene: a closed 10 x 8 x 3 m room, 20 spheres of radius
    0.2-1 m, one scanner at the room centre (5, 4, 1.5).  The room is closed, so
    every ray hits a surface and the cloud has exactly `n_points` points."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0])))
    dims = (10.0, 8.0, 3.0)
    scanner = np.array([5.0, 4.0, 1.5])
    rects, sid = _box_walls(*dims, 0)
    spheres = []
    while len(spheres) < 20:
        r = rng.uniform(0.2, 1.0)
        c = np.array([rng.uniform(r, dims[0] - r), rng.uniform(r, dims[1] - r), rng.uniform(r, dims[2] - r)])
        if np.linalg.norm(c - scanner) < r + 0.3:
            continue
        if any(np.linalg.norm(c - o[:3]) < r + o[3] for o in spheres):
            continue
        spheres.append(np.array([c[0], c[1], c[2], r, sid])); sid += 1
    colors = rng.integers(30, 226, size=(sid, 3)).astype(np.uint8)
    prims = Primitives(np.array(rects, dtype=np.float64), np.array(spheres), np.zeros((0, 7)),
                       np.zeros((0, 6)), colors)
    workers = _default_workers() if workers is None else workers
    caps = [np.zeros((0, 4))]
    gains = [np.ones(3)]
    xyz, rgb = _run_scans(seed, [scanner], n_points, prims, caps, gains, 100_000, workers)
    return Scene(xyz, rgb, scanner[None, :], ((0.0, 0.0, 0.0), dims),
                 np.array([[5.0, 4.0, 1.6]]), np.array([0]), name=f"room-s{seed}-n{n_points}")


def multiroom_scene(seed: int = 0, n_points: int = 20_000_000, n_scans: int = 4,
                    rooms_x: int = 4, rooms_y: int = 2, room_w: float = 10.0, room_d: float = 15.0,
                    height: float = 6.0, n_boxes: int = 48, n_cyl: int = 24,
                    gap_coverage: float = 0.2, workers: Optional[int] = None,
                    chunk_rays: int = 1_000_000,
                    progress: Optional[Callable[[str], None]] = None) -> Scene:
    """Multi-room, multi-scan scene.

    Default: 40 x 30 x 6 m split into eight 10 x 15 m rooms by interior walls
    (x = 10, 20, 30 and y = 15); each interior wall segment has one 1.2 x 2.2 m
    door; 48 floor boxes and 24 vertical cylinders; `n_scans` scanners at
    z = 1.5 in distinct rooms, `n_points / n_scans` points each, per-scan
    colour gains and 20 % occlusion gaps."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0])))
    X, Y, Z = rooms_x * room_w, rooms_y * room_d, height
    rects, sid = _box_walls(X, Y, Z, 0)
    # interior walls split into segments, each with one door
    door_w, door_h = 1.2, 2.2
    for i in range(1, rooms_x):
        x = i * room_w
        for j in range(rooms_y):
            y0, y1 = j * room_d, (j + 1) * room_d
            d0 = rng.uniform(y0 + 0.5, y1 - 0.5 - door_w)
            rects.append((0, x, y0, d0, 0.0, Z, sid))
            rects.append((0, x, d0 + door_w, y1, 0.0, Z, sid))
            rects.append((0, x, d0, d0 + door_w, door_h, Z, sid)); sid += 1
    for j in range(1, rooms_y):
        y = j * room_d
        for i in range(rooms_x):
            x0, x1 = i * room_w, (i + 1) * room_w
            d0 = rng.uniform(x0 + 0.5, x1 - 0.5 - door_w)
            rects.append((1, y, x0, d0, 0.0, Z, sid))
            rects.append((1, y, d0 + door_w, x1, 0.0, Z, sid))
            rects.append((1, y, d0, d0 + door_w, door_h, Z, sid)); sid += 1
    n_rooms = rooms_x * rooms_y
    room_centers = np.array([[(i + 0.5) * room_w, (j + 0.5) * room_d, 1.6]
                             for j in range(rooms_y) for i in range(rooms_x)])
    scan_rooms = rng.permutation(n_rooms)[: min(n_scans, n_rooms)]
    if n_scans > n_rooms:
        scan_rooms = np.concatenate([scan_rooms, rng.integers(0, n_rooms, n_scans - n_rooms)])
    c0 = room_centers[scan_rooms[0]]

    def near_orbit(x0, y0, x1, y1):
        # footprint distance range from the orbit centre of the first scanner's room
        dx = max(x0 - c0[0], 0.0, c0[0] - x1)
        dy = max(y0 - c0[1], 0.0, c0[1] - y1)
        dmin = np.hypot(dx, dy)
        dmax = max(np.hypot(px - c0[0], py - c0[1]) for px in (x0, x1) for py in (y0, y1))
        return dmin < 3.7 and dmax > 2.3

    scanners = []
    for r in scan_rooms:
        c = room_centers[r]
        scanners.append(np.array([c[0] + rng.uniform(-2.5, 2.5), c[1] + rng.uniform(-4.0, 4.0), 1.5]))
    scanners = np.array(scanners)

    def clear_of_scanners(x0, y0, x1, y1):
        for s in scanners:
            dx = max(x0 - s[0], 0.0, s[0] - x1)
            dy = max(y0 - s[1], 0.0, s[1] - y1)
            if np.hypot(dx, dy) < 0.6:
                return False
        return True

    boxes = []
    while len(boxes) < n_boxes:
        sx, sy = rng.uniform(0.3, 2.0, 2)
        h = rng.uniform(0.3, 2.5)
        x0 = rng.uniform(0.2, X - sx - 0.2)
        y0 = rng.uniform(0.2, Y - sy - 0.2)
        if not clear_of_scanners(x0, y0, x0 + sx, y0 + sy) or near_orbit(x0, y0, x0 + sx, y0 + sy):
            continue
        boxes.append((x0, y0, 0.0, x0 + sx, y0 + sy, h, sid)); sid += 1
    cyls = []
    while len(cyls) < n_cyl:
        r = rng.uniform(0.1, 0.5)
        h = rng.uniform(1.0, Z)
        cx = rng.uniform(r + 0.2, X - r - 0.2)
        cy = rng.uniform(r + 0.2, Y - r - 0.2)
        if not clear_of_scanners(cx - r, cy - r, cx + r, cy + r) or near_orbit(cx - r, cy - r, cx + r, cy + r):
            continue
        cyls.append((cx, cy, r, 0.0, h, sid)); sid += 1
    colors = rng.integers(30, 226, size=(sid, 3)).astype(np.uint8)
    prims = Primitives(np.array(rects, dtype=np.float64), np.zeros((0, 5)), np.array(boxes, dtype=np.float64),
                       np.array(cyls, dtype=np.float64), colors)
    caps = [_make_caps(np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 100 + k]))), gap_coverage)
            for k in range(n_scans)]
    grng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 99])))
    gains = [grng.normal(1.0, 0.05, 3) for _ in range(n_scans)]
    quota = [n_points // n_scans + (1 if k < n_points % n_scans else 0) for k in range(n_scans)]
    workers = _default_workers() if workers is None else workers
    xs, cs = [], []
    for k in range(n_scans):
        x, c = _run_scans(seed * 1000 + k, [scanners[k]], quota[k], prims, [caps[k]], [gains[k]],
                          chunk_rays, workers)
        xs.append(x); cs.append(c)
        if progress is not None:
            progress(f"scan {k + 1}/{n_scans}: {x.shape[0]} points")
    return Scene(np.concatenate(xs), np.concatenate(cs), scanners, ((0.0, 0.0, 0.0), (X, Y, Z)),
                 room_centers, scan_rooms, name=f"multiroom-s{seed}-n{n_points}-k{n_scans}")


def _cache_dir() -> str:
    return os.environ.get("LNR_SCENE_CACHE", "/tmp/lnr_scene_cache")


def scene_for_config(name: str, seed: int = 0, n_points: Optional[int] = None,
                     cache: bool = True, workers: Optional[int] = None,
                     progress: Optional[Callable[[str], None]] = None) -> Scene:
    """Named workloads.

    room     : 200k-point single-scan room (10 x 8 x 3 m, 20 spheres, 0.5 m cells)
    multiroom: 20M-point 4-scan multi-room scene (40 x 30 x 6 m, 1 m cells)
    large    : 100M points, 8 scans, same generator
    huge     : 300M points, 16 scans, 80 x 60 x 10 m (32 rooms)
    """
    params = {
        "room": dict(kind="room", n_points=200_000),
        "multiroom": dict(kind="multi", n_points=20_000_000, n_scans=4),
        "large": dict(kind="multi", n_points=100_000_000, n_scans=8),
        "huge": dict(kind="multi", n_points=300_000_000, n_scans=16, rooms_x=8, rooms_y=4, height=10.0),
    }[name]
    params = dict(params)
    if n_points is not None:
        params["n_points"] = n_points
    kind = params.pop("kind")
    key = hashlib.sha1(repr((name, seed, sorted(params.items()), 3)).encode()).hexdigest()[:16]
    path = os.path.join(_cache_dir(), f"{name}-{key}.npz")
    if cache and os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        return Scene(z["xyz"], z["rgb"], z["scanners"], (tuple(z["b0"]), tuple(z["b1"])), z["rooms"],
                     z["scan_rooms"], name=str(z["name"]))
    if kind == "room":
        sc = room_scene(seed, params["n_points"], workers=workers)
    else:
        sc = multiroom_scene(seed, workers=workers, progress=progress, **params)
    if cache:
        os.makedirs(_cache_dir(), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, xyz=sc.xyz, rgb=sc.rgb, scanners=sc.scanners, b0=np.array(sc.bounds[0]),
                 b1=np.array(sc.bounds[1]), rooms=sc.room_centers, scan_rooms=sc.scanner_rooms,
                 name=np.array(sc.name))
        os.replace(tmp, path)
    return sc
