"""Seeded U-Net weight blobs.

The trained weights of the paper are not available, so networks are
initialised from a seed: He-normal weights W ~ N(0, 2 / fan_in) with
fan_in = C_in * k * k, and zero biases (or, for tests, biases drawn from
U(-0.1, 0.1)).

Blob layout (little endian), one record per convolution:

    char[4]  magic "LNRU"
    u32      version (1; 2 when records carry a batch-norm flag)
    u32      L (levels), u32 in_channels, u32 out_channels, u32 widths[L]
    4L-1 records, in network order:
        u32 c_out, u32 c_in, u32 k
        version 2 only: u32 has_bn
        f32 weight[c_out * c_in * k * k]   (OIHW)
        f32 bias[c_out]
        if has_bn: f32 gamma[c_out], beta[c_out], mean[c_out], var[c_out], f32 eps

A batch-norm record means conv -> BN -> ReLU; loaders fold it into the
convolution (the paper places BN after each encoder convolution, used
as a training aid).

Network order: enc0a, enc0b, enc1a, enc1b, ..., enc{L-1}a, enc{L-1}b,
dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b, head.  Decoder level l takes the
concatenation [skip_l (w_l channels), upsampled (w_{l+1} channels)].
"""

from __future__ import annotations

import dataclasses
import struct
from typing import List, Sequence, Tuple

import numpy as np

MAGIC = b"LNRU"


@dataclasses.dataclass
class UNetSpec:
    widths: Tuple[int, ...]
    in_ch: int = 5
    out_ch: int = 3

    @property
    def levels(self) -> int:
        return len(self.widths)


def unet_layer_shapes(spec: UNetSpec) -> List[Tuple[str, int, int, int]]:
    """(name, c_out, c_in, k) for every convolution, in blob order."""
    w = spec.widths
    L = len(w)
    out = []
    for l in range(L):
        cin = spec.in_ch if l == 0 else w[l - 1]
        out.append((f"enc{l}a", w[l], cin, 3))
        out.append((f"enc{l}b", w[l], w[l], 3))
    for l in range(L - 2, -1, -1):
        out.append((f"dec{l}a", w[l], w[l] + w[l + 1], 3))
        out.append((f"dec{l}b", w[l], w[l], 3))
    out.append(("head", spec.out_ch, w[0], 1))
    return out


def make_unet_blob(widths: Sequence[int], seed: int = 0, bias: str = "zero",
                   in_ch: int = 5, out_ch: int = 3, batchnorm: bool = False) -> bytes:
    spec = UNetSpec(tuple(int(x) for x in widths), in_ch, out_ch)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 42])))
    parts = [MAGIC, struct.pack("<4I", 2 if batchnorm else 1, spec.levels, in_ch, out_ch),
             struct.pack(f"<{spec.levels}I", *spec.widths)]
    for name, co, ci, k in unet_layer_shapes(spec):
        fan_in = ci * k * k
        W = rng.normal(0.0, np.sqrt(2.0 / fan_in), size=(co, ci, k, k)).astype(np.float32)
        if bias == "zero":
            b = np.zeros(co, dtype=np.float32)
        elif bias == "uniform":
            b = rng.uniform(-0.1, 0.1, co).astype(np.float32)
        else:
            raise ValueError(bias)
        has_bn = batchnorm and name.startswith("enc")
        parts.append(struct.pack("<3I", co, ci, k))
        if batchnorm:
            parts.append(struct.pack("<I", 1 if has_bn else 0))
        parts += [W.tobytes(), b.tobytes()]
        if has_bn:
            gamma = rng.uniform(0.5, 1.5, co).astype(np.float32)
            beta = rng.uniform(-0.2, 0.2, co).astype(np.float32)
            mean = rng.uniform(-0.2, 0.2, co).astype(np.float32)
            var = rng.uniform(0.5, 2.0, co).astype(np.float32)
            parts += [gamma.tobytes(), beta.tobytes(), mean.tobytes(), var.tobytes(),
                      struct.pack("<f", 1e-5)]
    return b"".join(parts)
