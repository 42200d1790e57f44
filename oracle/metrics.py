"""Error metrics for the reconstructed image (oracle; test infrastructure).

max-abs = max over all output values of |y - y_ref|.
PSNR = 10 log10(peak^2 / MSE), with peak = max(y_ref) - min(y_ref) over the
frame: the networks here have random weights, so their output has no fixed
[0, 1] range and the reference's own spread is used as the peak.
"""

from __future__ import annotations

import numpy as np


def max_abs(y: np.ndarray, ref: np.ndarray) -> float:
    return float(np.max(np.abs(np.asarray(y, dtype=np.float64) - np.asarray(ref, dtype=np.float64))))


def psnr(y: np.ndarray, ref: np.ndarray) -> float:
    ref = np.asarray(ref, dtype=np.float64)
    mse = float(np.mean((np.asarray(y, dtype=np.float64) - ref) ** 2))
    peak = float(ref.max() - ref.min())
    if mse == 0.0:
        return float("inf")
    return 10.0 * np.log10(peak * peak / mse)
