"""CPU oracle for the per-frame rendering path of "Real-time Neural Rendering
of LiDAR Point Clouds" (arXiv 2502.11618).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of what the method computes, used to check the HIP path.  Only
the test suite, the package smoke check and the CPU-baseline leg of the bench
may import it; the product path never does and shares no code with it.

Arithmetic conventions:
  * the geometric stages (partition, culling, projection/z-buffer, resolve,
    min-pool pyramid, depth filter) are written in IEEE binary32 in an
    explicit operation order with no fused multiply-add (numpy float32
    element-wise operations round after every operation), so the result is
    a single well-defined bit pattern;
  * the U-Net forward pass is evaluated in float64.

Modules:
  grid          uniform-grid partition and conservative frustum culling
  render        1x1 point projection into a z-buffer and RGBDA resolve
  depth_filter  min-pool pyramid and hierarchical depth filter
  unet          weight-blob parser and float64 U-Net forward pass
  metrics       max-abs error and PSNR

Parity status per function is stated in each module header.
"""
