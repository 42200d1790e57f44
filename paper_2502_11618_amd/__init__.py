"""MI355X (gfx950) per-frame rendering path of "Real-time Neural Rendering of
LiDAR Point Clouds" (arXiv 2502.11618): grid culling, 1x1 point projection
into RGBDA, hierarchical min-pool depth filter and U-Net reconstruction, as a
C-ABI library of hand-written HIP kernels (liblnr.so) with a ctypes binding.

The binding (paper_2502_11618_amd.lnr) loads liblnr.so on first use of any of
its names and fails loudly if the library is not built; importing the
package itself does not load it, so `paper_2502_11618_amd.build` can run on
a fresh checkout.
"""

import importlib


_SUBMODULES = ("lnr", "build")


def __getattr__(name):
    if name.startswith("__"):
        raise AttributeError(name)
    if name in _SUBMODULES:
        return importlib.import_module(f"{__name__}.{name}")
    return getattr(importlib.import_module(__name__ + ".lnr"), name)
