"""MI355X (gfx950) per-frame rendering path of "Real-time Neural Rendering of
LiDAR Point Clouds" (arXiv 2502.11618): grid culling, 1x1 point projection
into RGBDA, hierarchical min-pool depth filter and U-Net reconstruction, as a
C-ABI library of hand-written HIP kernels (liblnr.so) with a ctypes binding.

Importing the package loads liblnr.so and fails loudly if it is not built.
"""

from .lnr import *  # noqa: F401,F403
from .lnr import (  # noqa: F401
    Cloud, Context, Image, LnrError, UNet, camera_struct, lnr_camera, lnr_image, LIB_PATH,
)
