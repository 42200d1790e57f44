"""The bench's roofline arithmetic against counts that do not come from its
own formulas: the U-Net flops it divides by (every 3x3 convolution of the
1080p network, and the four executed by Winograd) against the multiply-adds
the float64 oracle's forward pass runs (pinned by a shape count in
test_oracle_unet.py), and the executed Winograd work against a count of the
2x2 output blocks and transform positions of a small image."""

import numpy as np

import bench
import synth
from oracle import unet as U


def test_bench_unet_flops_equal_the_oracle_count():
    widths = (32, 64, 128, 256)
    net = U.parse_blob(synth.make_unet_blob(widths, seed=0))
    H, W = 1080, 1920
    shapes = bench.conv_shapes(widths, H, W, 8)
    flops = sum(2.0 * h * w * co * 9 * ci for (_, h, w, co, ci) in shapes) + 2.0 * H * W * 3 * widths[0]
    assert flops == U.flops_per_pixel(net) * H * W
    assert abs(flops - 675.2e9) < 0.05e9  # the figure the roofline quotes
    assert [n for (n, *_) in shapes] == ["conv/enc0a", "conv/enc0b", "conv/enc1a", "conv/enc1b", "conv/enc2a",
                                         "conv/enc2b", "conv/enc3a", "conv/enc3b", "conv/dec2a", "conv/dec2b",
                                         "conv/dec1a", "conv/dec1b", "conv/dec0a", "conv/dec0b"]


def test_winograd_executed_flops_count_blocks_and_positions():
    """F(2x2, 3x3): one 16-position product per 2x2 output block (ragged
    blocks included) and channel pair; enumerated on a small odd-sized layer
    and compared with the formula the bench uses for conv/dec0a (50.96 GFLOP
    at 1080p)."""
    h, w, ci, co = 7, 11, 3, 5
    blocks = {(y // 2, x // 2) for y in range(h) for x in range(w)}
    products = len(blocks) * 16 * ci * co
    assert 2.0 * ((h + 1) // 2) * ((w + 1) // 2) * 16 * ci * co == 2.0 * products
    shapes = dict((n, (hh, ww, c_o, c_i)) for (n, hh, ww, c_o, c_i) in bench.conv_shapes((32, 64, 128, 256), 1080,
                                                                                         1920, 8))
    hh, ww, c_o, c_i = shapes["conv/dec0a"]
    assert 2.0 * ((hh + 1) // 2) * ((ww + 1) // 2) * 16 * c_i * c_o == 50960793600.0
