"""Pins of the oracle's BF16 halo definitions: the conversion against
PyTorch's float32 -> bfloat16 cast (round to nearest, ties to even), the
half-ulp bound, exact ties, values BF16 represents exactly, special values;
the shared planes of a slab against the cell-layer geometry."""

import numpy as np
import pytest
import torch

from oracle import halo
from oracle.paw import PAWOperator
from workloads.configs import custom_system


def test_bf16_matches_library_cast():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(20000), rng.standard_normal(2000) * 1e30,
                        rng.standard_normal(2000) * 1e-30]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(halo.to_bf16_bits(x), want)


def test_bf16_half_ulp_bound_and_exact_values():
    rng = np.random.default_rng(2)
    x = rng.standard_normal(50000).astype(np.float32)
    y = halo.from_bf16_bits(halo.to_bf16_bits(x))
    assert np.all(np.abs(y - x) <= np.abs(x) * 2.0 ** -8)
    # values with 8 significant bits are exact
    z = (rng.integers(-255, 256, 1000) * 2.0 ** rng.integers(-20, 20, 1000)).astype(np.float32)
    np.testing.assert_array_equal(halo.from_bf16_bits(halo.to_bf16_bits(z)), z)


def test_bf16_ties_and_specials():
    # 1 + 2^-8 lies halfway between 1 and 1 + 2^-7: ties to even (1)
    t = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8)], dtype=np.float32)
    np.testing.assert_array_equal(halo.from_bf16_bits(halo.to_bf16_bits(t)),
                                  np.array([1.0, 1 + 2 * 2.0 ** -7, -1.0], dtype=np.float32))
    s = np.array([0.0, -0.0, np.inf, -np.inf, np.float32(3.4e38)], dtype=np.float32)
    back = halo.from_bf16_bits(halo.to_bf16_bits(s))
    assert back[0] == 0 and np.signbit(back[1]) and back[2] == np.inf and back[3] == -np.inf
    assert back[4] == np.inf                                   # rounds past the largest BF16
    assert np.isnan(halo.from_bf16_bits(halo.to_bf16_bits(np.array([np.nan], np.float32))))[0]


def test_shared_planes_and_pack_layout():
    s = custom_system((3, 2, 4), (3.0, 2.0, 4.0), 3, 5)
    op = PAWOperator(s)
    p, (Gx, Gy, Gz) = op.mesh.p, op.mesh.G
    assert halo.shared_planes(op, 1, 3) == (p, 3 * p)
    assert halo.shared_planes(op, 2, 4) == (2 * p, 0)            # periodic wrap
    # plane rows are exactly the DOFs with that z index, (gy, gx) row-major
    rows = halo.plane_rows(op, 5)
    I = np.arange(op.mesh.M)
    np.testing.assert_array_equal(np.sort(rows), I[(I // (Gx * Gy)) == 5])
    assert rows[1] - rows[0] == 1 and rows[Gx] - rows[0] == Gx
    Y = np.random.default_rng(3).standard_normal((op.mesh.M, 5)).astype(np.float32)
    buf = halo.pack(op, Y, 1, 3)
    assert buf.shape == (2, Gx * Gy, 5) and buf.dtype == np.uint16
    out = halo.unpack_add(op, buf, Y, 1, 3)
    others = np.setdiff1d(I, np.concatenate([halo.plane_rows(op, p), halo.plane_rows(op, 3 * p)]))
    np.testing.assert_array_equal(out[others], Y[others])
    r = halo.plane_rows(op, p)
    np.testing.assert_allclose(out[r], 2 * Y[r], rtol=2.0 ** -7)
