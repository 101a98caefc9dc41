"""Reduced-precision halo exchange of a slab decomposition in the oracle
(TEST INFRASTRUCTURE).

The paper's reduced-precision inter-processor communication (the
"Reduced precision inter-processor communication" paragraph and the figure
on BF16 communication): after the local operator action, the partial sums on
the node planes a processor shares with its neighbour are sent in BF16 and
cast back to FP32, where the receiving processor adds them to its own.

For a slab of cell layers [kz0, kz1) along z of the periodic mesh, the shared
node planes are gz = kz0 p and gz = (kz1 p) mod Gz.  ``pack`` gives, for both
planes in that order, the BF16 bits of the FP32 values of every node of the
plane (node I = gx + Gx (gy + Gy gz), row-major over (gy, gx)) and column;
``unpack_add`` adds the BF16 values, cast to FP32, to an FP32 block in FP32
arithmetic.

BF16 is the upper half of an IEEE binary32 number; the conversion rounds the
dropped 16 bits to nearest, ties to even, and keeps NaNs NaN.
"""

from __future__ import annotations

import numpy as np


def to_bf16_bits(x):
    """BF16 bits (uint16) of float32 values: round to nearest, ties to even."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    upper = u >> np.uint64(16)
    lower = u & np.uint64(0xFFFF)
    half = np.uint64(0x8000)
    # round up when the dropped part is above half, or exactly half with an odd kept part
    up = (lower > half) | ((lower == half) & ((upper & np.uint64(1)) == np.uint64(1)))
    r = upper + up.astype(np.uint64)
    nan = np.isnan(x)
    r = np.where(nan, upper | np.uint64(0x40), r)
    return r.astype(np.uint16)


def from_bf16_bits(b):
    """float32 values of BF16 bits (exact: BF16 is a subset of binary32)."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << np.uint32(16)).view(np.float32)


def shared_planes(op, kz0, kz1):
    """Global z node indices of the slab's two shared planes."""
    p = op.mesh.p
    Gz = op.mesh.G[2]
    return (kz0 * p) % Gz, (kz1 * p) % Gz


def plane_rows(op, gz):
    """DOF indices of node plane gz, ordered (gy, gx) row-major."""
    Gx, Gy, _ = op.mesh.G
    gy, gx = np.meshgrid(np.arange(Gy), np.arange(Gx), indexing="ij")
    return (gx + Gx * (gy + Gy * gz)).ravel()


def pack(op, Y, kz0, kz1):
    """BF16 bits of Y (float32 [ndof][ncols]) on the two shared planes: [2][Gx Gy][ncols]."""
    Y = np.asarray(Y, dtype=np.float32)
    return np.stack([to_bf16_bits(Y[plane_rows(op, gz)]) for gz in shared_planes(op, kz0, kz1)])


def unpack_add(op, buf, Y, kz0, kz1):
    """Y (float32) with the BF16 values of buf added on the two shared planes."""
    out = np.array(Y, dtype=np.float32, copy=True)
    for t, gz in enumerate(shared_planes(op, kz0, kz1)):
        rows = plane_rows(op, gz)
        out[rows] = out[rows] + from_bf16_bits(buf[t])
    return out
