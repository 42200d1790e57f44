"""Pins of the error metrics (CPU only)."""

import numpy as np

from oracle import metrics as M


def test_max_abs_and_psnr_closed_forms():
    ref = np.array([0.0, 1.0, 2.0, 3.0])
    y = ref + np.array([0.0, 0.1, -0.1, 0.0])
    assert abs(M.max_abs(y, ref) - 0.1) < 1e-15
    # peak = 3, MSE = 0.02/4 = 0.005 -> 10 log10(9 / 0.005)
    assert abs(M.psnr(y, ref) - 10 * np.log10(9 / 0.005)) < 1e-9
    assert M.psnr(ref, ref) == float("inf")
