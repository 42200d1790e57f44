"""The seeded scene generators hold the workload shapes the benchmarks name
(CPU): the largest configuration's building is 80 x 60 x 10 m of 32 rooms
scanned from 16 positions in distinct rooms, each scan giving an equal share
of the points, every point on the building's surfaces or inside it."""

import numpy as np

import synth


def test_largest_scene_layout():
    calls = []
    sc = synth.scene_for_config("huge", seed=0, n_points=32_000, cache=False, workers=1, progress=calls.append)
    assert sc.n == 32_000 and sc.xyz.shape == (32_000, 3) and sc.rgb.shape == (32_000, 3)
    assert sc.xyz.dtype == np.float32 and sc.rgb.dtype == np.uint8
    assert sc.bounds == ((0.0, 0.0, 0.0), (80.0, 60.0, 10.0))
    lo, hi = sc.xyz.min(axis=0), sc.xyz.max(axis=0)
    assert np.all(lo >= -1e-4) and np.all(hi <= np.array([80.0, 60.0, 10.0]) + 1e-4)
    assert len(sc.scanners) == 16 and len(sc.room_centers) == 32
    assert len(set(np.asarray(sc.scanner_rooms).tolist())) == 16
    assert calls == [f"scan {k + 1}/16: 2000 points" for k in range(16)]
    again = synth.scene_for_config("huge", seed=0, n_points=32_000, cache=False, workers=1)
    assert np.array_equal(sc.xyz, again.xyz) and np.array_equal(sc.rgb, again.rgb)
