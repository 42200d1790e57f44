"""Pinhole cameras for the synthetic workloads.

The paper does not fix a camera model.  The cameras here are pinholes with a
*horizontal* field of view, square pixels, principal point (W/2, H/2) and
OpenCV axes (x right, y down, z forward; world z is up).  The 3x4 projection
P = K [R | -R c] is formed in float64 and rounded to float32 once; the
renderer and its checkers both consume those same twelve floats.  The third
row of P gives the camera-space depth of a world point.
"""

from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

NEAR = 0.1
FAR = 1000.0


@dataclasses.dataclass
class Camera:
    P: np.ndarray      # float32 [12], row-major 3x4
    width: int
    height: int
    z_near: float = NEAR
    z_far: float = FAR


def look_at(eye, target, width: int, height: int, fov_deg: float,
            z_near: float = NEAR, z_far: float = FAR) -> Camera:
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    fwd = target - eye
    fwd /= np.linalg.norm(fwd)
    up = np.array([0.0, 0.0, 1.0])
    right = np.cross(fwd, up)
    if np.linalg.norm(right) < 1e-9:  # looking straight up or down
        right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    down = np.cross(fwd, right)
    R = np.stack([right, down, fwd])
    f = (width / 2.0) / np.tan(np.deg2rad(fov_deg) / 2.0)
    K = np.array([[f, 0.0, width / 2.0], [0.0, f, height / 2.0], [0.0, 0.0, 1.0]])
    Rt = np.concatenate([R, (-R @ eye)[:, None]], axis=1)
    P = (K @ Rt).astype(np.float32).reshape(12)
    return Camera(P, int(width), int(height), float(z_near), float(z_far))


def room_cameras(scene, n: int = 16, seed: int = 0, width: int = 256, height: int = 256,
                 fov_deg: float = 70.0) -> List[Camera]:
    """Seeded poses inside the single-scan room, clear of walls by 0.3 m and of the
    spheres, each looking at a random point of the cloud at least 1 m away.
    Poses away from the scanner make background leakage visible."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7])))
    (x0, y0, z0), (x1, y1, z1) = scene.bounds
    xyz = scene.xyz
    cams = []
    while len(cams) < n:
        eye = np.array([rng.uniform(x0 + 0.3, x1 - 0.3), rng.uniform(y0 + 0.3, y1 - 0.3),
                        rng.uniform(z0 + 0.3, z1 - 0.3)])
        # keep out of solid objects: nearest cloud point must be >= 0.3 m away
        if np.min(np.sum((xyz[:: max(1, xyz.shape[0] // 20000)] - eye) ** 2, axis=1)) < 0.09:
            continue
        tgt = xyz[rng.integers(0, xyz.shape[0])].astype(np.float64)
        if np.linalg.norm(tgt - eye) < 1.0:
            continue
        cams.append(look_at(eye, tgt, width, height, fov_deg))
    return cams


def orbit_path(scene, n_frames: int = 120, width: int = 1920, height: int = 1080,
               fov_deg: float = 90.0, radius: float = 3.0) -> List[Camera]:
    """Camera path: n frames on a circle of radius 3 m around the centre of the
    first scanner's room at z = 1.6, frame i at angle 2*pi*i/n, looking at the
    room centre turned by +20 degrees of yaw and -10 degrees of pitch."""
    c = scene.room_centers[int(scene.scanner_rooms[0])].astype(np.float64)
    cams = []
    for i in range(n_frames):
        th = 2.0 * np.pi * i / n_frames
        eye = c + radius * np.array([np.cos(th), np.sin(th), 0.0])
        to_c = c - eye
        yaw = np.arctan2(to_c[1], to_c[0]) + np.deg2rad(20.0)
        pitch = np.deg2rad(-10.0)
        d = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
        cams.append(look_at(eye, eye + d, width, height, fov_deg))
    return cams


def random_walk_path(scene, n_frames: int, seed: int, width: int, height: int,
                     fov_deg: float = 90.0, step: float = 0.05) -> List[Camera]:
    """A viewer session: start at a random point at z = 1.6 inside the scene, move
    `step` metres along the heading per frame, turn the yaw by N(0, 3 degrees)
    per frame and reflect off the outer walls."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 11])))
    (x0, y0, _), (x1, y1, _) = scene.bounds
    pos = np.array([rng.uniform(x0 + 1, x1 - 1), rng.uniform(y0 + 1, y1 - 1), 1.6])
    yaw = rng.uniform(0, 2 * np.pi)
    cams = []
    for _ in range(n_frames):
        d = np.array([np.cos(yaw), np.sin(yaw), 0.0])
        cams.append(look_at(pos, pos + d, width, height, fov_deg))
        nxt = pos + step * d
        if not (x0 + 0.5 < nxt[0] < x1 - 0.5):
            yaw = np.pi - yaw
        if not (y0 + 0.5 < nxt[1] < y1 - 0.5):
            yaw = -yaw
        pos = pos + step * np.array([np.cos(yaw), np.sin(yaw), 0.0])
        yaw += np.deg2rad(rng.normal(0.0, 3.0))
    return cams
