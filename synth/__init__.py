"""Seeded synthetic inputs shared by the oracle's tests, the GPU tests and the bench.

This package only *makes inputs*: coloured point clouds shaped like static
LiDAR scans, pinhole cameras, and U-Net weight blobs.  It contains none of the
rendering method's arithmetic (no projection, z-buffer, depth filter or
convolution), so the CPU oracle and the HIP path can both consume its output
without sharing any of the method's code.
"""

from .scene import (  # noqa: F401
    Scene,
    room_scene,
    multiroom_scene,
    scene_for_config,
)
from .camera import (  # noqa: F401
    Camera,
    look_at,
    room_cameras,
    orbit_path,
    random_walk_path,
)
from .unet_weights import (  # noqa: F401
    UNetSpec,
    make_unet_blob,
    unet_layer_shapes,
)
